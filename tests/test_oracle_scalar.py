"""Pins of the oracle's scalar part (coefficients, degree, occupations, mu,
eigenvalues, bounds) against closed forms, library routines and brute force.
CPU only."""
import json
import math
import os

import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest
import scipy.fft
import scipy.special

from oracle import chebyshev as cb

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def nodes(lo, hi, n):
    s, t = cb.scale_shift(lo, hi)
    k = np.arange(n)
    return np.cos(np.pi * (k + 0.5) / n) / s + t


def test_coefficients_are_a_dct_ii():
    # Eq. 5 is the (unnormalised) DCT-II of f at the Chebyshev nodes, over n.
    f = lambda x: np.exp(np.sin(3 * x)) + x ** 3
    for n in (1, 2, 7, 64, 333):
        c = cb.cheb_coeffs(f, -1.3, 2.0, n)
        ref = scipy.fft.dct(f(nodes(-1.3, 2.0, n)), type=2) / n
        assert np.max(np.abs(c - ref)) < 1e-13 * max(1, np.max(np.abs(ref)))


def test_coefficients_of_a_chebyshev_polynomial():
    # f = T_m(x~) gives c_j = delta_jm for m >= 1 and c_0 = 2 for m = 0
    # (discrete orthogonality of the cosines at the nodes; c_0 is halved in Eq. 1).
    lo, hi = -0.4, 3.0
    s, t = cb.scale_shift(lo, hi)
    n = 40
    for m in (0, 1, 5, 17, 39):
        f = lambda x, m=m: np.cos(m * np.arccos(np.clip(s * (x - t), -1, 1)))
        c = cb.cheb_coeffs(f, lo, hi, n)
        ref = np.zeros(n)
        ref[m] = 2.0 if m == 0 else 1.0
        assert np.max(np.abs(c - ref)) < 1e-13


def test_coefficients_of_exponential_are_bessel():
    # e^{a x} = I_0(a) + 2 sum_j I_j(a) T_j(x); the interpolant's aliasing is
    # below 1e-15 for n = 40, a = 1.5.
    a, n = 1.5, 40
    c = cb.cheb_coeffs(lambda x: np.exp(a * x), -1.0, 1.0, n)
    ref = 2 * scipy.special.iv(np.arange(n), a)
    assert np.max(np.abs(c - ref)) < 1e-14


def test_coefficients_of_inverse_are_geometric():
    # 1/(b - x) = sum' 2 r^j / sqrt(b^2 - 1) T_j(x), r = b - sqrt(b^2 - 1);
    # aliasing error of the n-point interpolant is ~ r^(2n-j).
    bb, n = 1.7, 60
    r = bb - math.sqrt(bb * bb - 1)
    c = cb.cheb_coeffs(lambda x: 1.0 / (bb - x), -1.0, 1.0, n)
    j = np.arange(n)
    ref = 2 * r ** j / math.sqrt(bb * bb - 1)
    alias = 4 * r ** (2 * n - j) / math.sqrt(bb * bb - 1) / (1 - r ** (2 * n))
    assert np.all(np.abs(c - ref) <= alias + 5e-15)


def test_interpolates_at_the_nodes_and_matches_numpy_chebval():
    f = lambda x: np.tanh(4 * x) + 0.1 * x
    lo, hi, n = -2.0, 1.5, 31
    c = cb.cheb_coeffs(f, lo, hi, n)
    s, t = cb.scale_shift(lo, hi)
    x = nodes(lo, hi, n)
    assert np.max(np.abs(cb.cheb_eval(c, s * (x - t)) - f(x))) < 1e-14
    xs = np.linspace(-1, 1, 101)
    c2 = c.copy()
    c2[0] *= 0.5
    assert np.max(np.abs(cb.cheb_eval(c, xs) - npc.chebval(xs, c2))) < 1e-13


def test_occupations():
    mu, kT = -0.3, 0.01
    e = np.linspace(-0.5, -0.1, 41)
    fe = cb.occ_erfc(e, mu, kT)
    assert abs(cb.occ_erfc(mu, mu, kT) - 0.5) < 1e-16
    assert np.max(np.abs(fe + cb.occ_erfc(2 * mu - e, mu, kT) - 1)) < 1e-15
    assert np.all(np.diff(fe) <= 0)
    fd = cb.occ_fermi_dirac(e, mu, kT)
    ref = np.array([1.0 / (1.0 + math.exp((x - mu) / kT)) for x in e])
    assert np.max(np.abs(fd - ref)) < 1e-15


def test_degree_is_monotone_and_meets_the_threshold():
    f = lambda e: cb.occ_erfc(e, 0.0, 0.05)
    prev = 0
    for tol in (1e-3, 1e-5, 1e-7, 1e-9):
        m = cb.degree(f, -1.0, 1.0, tol)
        assert m >= prev and m % 8 == 0
        assert cb.fit_error(f, -1.0, 1.0, m) < tol
        if m > 8:
            assert cb.fit_error(f, -1.0, 1.0, m - 8) >= tol
        prev = m


def test_degree_consistent_with_paper_inverse_example():
    # Sec. "Scaling with matrix size and sparsity" / "Parallel scaling": the
    # inverse of matrices with eigenvalues in [0.1, 1.1] (condition number 11)
    # needed an automatically chosen degree of 60.  The paper's threshold is
    # not printed; at a threshold near double precision our Eq. 7 search
    # lands in the same place.
    g = json.load(open(os.path.join(GOLDEN, "paper_inverse_degree.json")))
    m = cb.degree(cb.power_fn(-1.0), g["eig_lo"], g["eig_hi"], g["tol_fit_reading"])
    assert abs(m - g["n_pl_paper"]) <= g["band"]


def test_penalty_terms_consistent_with_paper_accuracy_degrees():
    # Sec. "Accuracy" (inverse of 6000-row matrices, degrees chosen with the
    # alpha = -200 penalty of Eq. 6): the smallest degree the paper reports,
    # 60, is where Eq. 6 becomes trustworthy on 6000 rows in reading R7,
    # while x^-1 itself needs far fewer terms at small condition numbers
    g = json.load(open(os.path.join(GOLDEN, "paper_accuracy_inverse_degrees.json")))
    m = cb.penalty_degree(g["n_rows"])
    assert abs(m - g["n_pl_min_paper"]) <= g["band"]
    assert cb.penalty_valid(m, g["n_rows"]) and not cb.penalty_valid(m - 8, g["n_rows"])
    assert cb.degree(cb.power_fn(-1.0), 1.0, 1.5, 1e-12) < g["n_pl_min_paper"] // 2


def diag_moments(lam, n_pl):
    th = np.arccos(np.clip(lam, -1, 1))
    return np.array([np.sum(np.cos(k * th)) for k in range(n_pl)])


def test_electron_count_and_mu_bisection_on_a_known_spectrum():
    # Diagonal M~ with eigenvalues lam: Tr T_k = sum_i cos(k arccos lam_i), so
    # N(mu) from the moments is sum_i p(lam_i); mu must solve the exact
    # occupation sum to within the polynomial error.
    rng = np.random.default_rng(1)
    lo, hi, kT = -1.0, 1.0, 0.05
    lam = np.sort(rng.uniform(-0.95, 0.95, 200))
    n_pl = cb.degree(lambda e: cb.occ_erfc(e, 0.0, kT), lo, hi, 1e-12)
    t = diag_moments(lam, n_pl)
    target = 77.0
    mu, it = cb.bisect_mu(t, lo, hi, kT, target, 1e-11)
    exact = np.sum(cb.occ_erfc(lam, mu, kT))
    assert abs(exact - target) < 200 * 1e-12 + 1e-10
    assert it > 5


def test_eigenvalues_from_moments_on_designed_spectrum():
    # Eigenvalues spaced far apart compared to the occupation width are found
    # to within a small fraction of that width.
    lam = np.linspace(-0.8, 0.8, 33)
    width = 8e-3  # spacing 0.05: still many widths apart, at a quarter of the degree
    lo, hi = -1.0, 1.0
    n_pl = cb.degree(lambda e: cb.occ_erfc(e, 0.0, width), lo, hi, 1e-10, m_max=6000)
    t = diag_moments(lam, n_pl)
    ev = cb.eigenvalues_from_moments(t, lo, hi, width, -0.31, 0.49)
    ref = lam[(lam >= -0.31) & (lam <= 0.49)]
    assert ev.shape == ref.shape
    assert np.max(np.abs(ev - ref)) < 1e-3 * width


def test_penalty_function_signs():
    # Eq. 6 with alpha < 0: a spectrum inside the bounds gives ~0, one below
    # the lower bound a large positive trace, one above the upper a negative.
    f = cb.penalty_fn(-200.0, -1.0, 1.0)
    assert abs(f(np.array([0.0]))[0]) < 1e-80
    assert f(np.array([-1.01]))[0] > 1.0
    assert f(np.array([1.01]))[0] < -1.0


def test_gershgorin_contains_the_spectrum_and_is_brute_force():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((30, 30))
    A = A + A.T
    lo, hi = cb.gershgorin(A)
    R = [sum(abs(A[i, j]) for j in range(30) if j != i) for i in range(30)]
    assert lo == pytest.approx(min(A[i, i] - R[i] for i in range(30)), abs=1e-12)
    assert hi == pytest.approx(max(A[i, i] + R[i] for i in range(30)), abs=1e-12)
    w = np.linalg.eigvalsh(A)
    assert lo <= w[0] and w[-1] <= hi


def test_lanczos_with_full_basis_is_exact():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((25, 25))
    A = A + A.T
    w = np.linalg.eigvalsh(A)
    tmin, tmax, rmin, rmax = cb.lanczos_extremes(lambda x: A @ x, 25, 25)
    assert abs(tmin - w[0]) < 1e-10 and abs(tmax - w[-1]) < 1e-10


def test_homo_lumo_on_designed_spectrum():
    # Levels 0.05 apart (over 6 widths): eigenvalues N_h = ceil(N_e) and
    # N_h + 1 come out to a small fraction of the width; past either end of
    # the spectrum the estimate is NaN.
    lam = np.linspace(-0.8, 0.8, 33)
    kT = 8e-3
    lo, hi = -1.0, 1.0
    n_pl = cb.degree(lambda e: cb.occ_erfc(e, 0.0, kT), lo, hi, 1e-10, m_max=6000)
    t = diag_moments(lam, n_pl)
    for n_e, nh in ((12, 12), (11.3, 12), (12.0000000001, 12), (1, 1), (32, 32)):
        homo, lumo = cb.homo_lumo_from_moments(t, lo, hi, kT, n_e)
        assert abs(homo - lam[nh - 1]) < 1e-3 * kT, (n_e, homo)
        assert abs(lumo - lam[nh]) < 1e-3 * kT, (n_e, lumo)
    homo, lumo = cb.homo_lumo_from_moments(t, lo, hi, kT, 33)
    assert abs(homo - lam[32]) < 1e-3 * kT and math.isnan(lumo)
    homo, lumo = cb.homo_lumo_from_moments(t, lo, hi, kT, 0)
    assert math.isnan(homo) and abs(lumo - lam[0]) < 1e-3 * kT
