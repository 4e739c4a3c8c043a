"""Pins of the energy check of Sec. "Fermi Operator Expansion" in the oracle:
E = Tr(K' H') from the moments of the chain (chebyshev.energy_from_moments)
against an explicit product of the oracle's own K' and H' on a sparse
(truncated) pattern, against sum_i f(e_i) e_i from a diagonalisation on a
dense pattern, and the width adaptation against decisions taken from exact
eigenvalues.  CPU only."""
import numpy as np
import pytest

from oracle import chebyshev as cb
from oracle import pipeline as opl
from oracle.csr import Csr, chebyshev
from workloads import generator as g


def test_energy_from_moments_equals_trace_of_product_on_truncated_pattern():
    # the truncated chain keeps the diagonal exactly, so the moment formula is
    # an identity for Tr(p(H~') H') even where p(H~') is only approximate
    s = g.make_system(40, 4, 4.6, 6.2, seed=3)
    H = opl.BlockMat(s.pat_h.nb, s.b, s.pat_h.row_ptr, s.pat_h.col_idx, s.H)
    P = opl.BlockMat(s.pat_k.nb, s.b, s.pat_k.row_ptr, s.pat_k.col_idx)
    lo, hi = -3.0, 0.2
    Hc = H.csr()
    K = P.pattern_csr()
    n_pl = 45
    c = cb.cheb_coeffs(lambda e: cb.occ_erfc(e, -1.0, 0.05), lo, hi, n_pl)
    acc, _ = chebyshev(opl.scaled(Hc, lo, hi), K, n_pl, c[None, :])
    _, mom = chebyshev(opl.scaled(Hc, lo, hi), K, n_pl + 1, None)
    Kp = K.with_values(acc[0]).dense()
    e_direct = float(np.sum(Kp * Hc.dense().T))
    assert abs(cb.energy_from_moments(c, mom, lo, hi) - e_direct) < 1e-10 * max(1.0, abs(e_direct))


def dense_system(eps, seed, b=1):
    """H, S (b = 1, dense pattern) with S^-1/2 H S^-1/2 having eigenvalues eps."""
    rng = np.random.default_rng(seed)
    n = eps.size
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * eps) @ Q.T
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    sv = rng.uniform(0.8, 1.25, n)
    Sh = (V * np.sqrt(sv)) @ V.T
    S = (V * sv) @ V.T
    H = Sh @ A @ Sh
    rp = np.arange(0, n * n + 1, n)
    ci = np.tile(np.arange(n), n)
    mk = lambda M: opl.BlockMat(n, 1, rp, ci, M.reshape(-1, 1, 1))
    return mk(H), mk(S), opl.BlockMat(n, 1, rp, ci)


def exact_energy(eps, n_e, kT):
    """E = sum_i f(e_i; mu) e_i with mu solving sum_i f = n_e (bisection)."""
    a, b = eps.min() - 50 * kT, eps.max() + 50 * kT
    for _ in range(200):
        m = 0.5 * (a + b)
        if np.sum(cb.occ_erfc(eps, m, kT)) < n_e:
            a = m
        else:
            b = m
    mu = 0.5 * (a + b)
    return float(np.sum(cb.occ_erfc(eps, mu, kT) * eps))


def test_energy_from_moments_matches_diagonalisation_on_dense_pattern():
    eps = np.concatenate([np.linspace(-1.0, -0.4, 14), np.linspace(0.05, 0.7, 16)])
    H, S, P = dense_system(eps, 1)
    for kT in (0.04, 0.1):
        _, info = opl.fermi_operator(H, S, P, 14.0, kT, h_bounds=(-1.1, 0.8), adapt_kt=True,
                                     tol_energy=1e9, tol_fit=1e-11)
        assert info["kt_halvings"] == 0
        # bar: mu is searched to |N - N_e| <= 1e-8 N_e, which moves E by about
        # |mu| 1e-8 N_e ~ 2e-8, plus the fit errors; a dropped term, a wrong
        # sign or a wrong shift changes E by O(1)
        assert abs(info["energy"] - exact_energy(eps, 14.0, kT)) < 1e-6
        assert abs(info["energy_wide"] - exact_energy(eps, 14.0, 1.25 * kT)) < 1e-6


def test_width_adaptation_follows_exact_energies():
    # gap 0.2 around the Fermi level: a wide occupation mixes the two sides
    # and E(kT) - E(1.25 kT) shrinks as kT is halved; the number of halvings
    # the oracle takes from its moments is the one the exact eigenvalues give
    eps = np.concatenate([np.linspace(-0.9, -0.1, 12), np.linspace(0.1, 0.8, 12)])
    H, S, P = dense_system(eps, 2)
    tol = 1e-4
    kT = 0.2
    expected = 0
    while True:
        d = abs(exact_energy(eps, 12.0, kT) - exact_energy(eps, 12.0, 1.25 * kT))
        assert abs(d - tol) > 0.2 * tol  # the decision is not at the threshold
        if d <= tol:
            break
        kT *= 0.5
        expected += 1
    assert expected == 3
    _, info = opl.fermi_operator(H, S, P, 12.0, 0.2, h_bounds=(-1.0, 0.9), adapt_kt=True,
                                 tol_energy=tol, tol_fit=1e-11, max_kt_halvings=6)
    assert info["kt_halvings"] == expected
    assert info["kT"] == pytest.approx(0.2 * 0.5 ** expected)
    assert abs(info["energy"] - exact_energy(eps, 12.0, info["kT"])) < 1e-6
