"""Pins of the oracle's bound handling: the Eq. 7 fit-error grid (reading R8),
the Eq. 6 check with its side rule and widening loop (reading R7), and the
truncation order of the orthogonal frame and of the post-transform on a
sparse pattern where truncation changes the result.  CPU only."""
import math

import numpy as np
import numpy.polynomial.chebyshev as npcheb
import pytest

from oracle import chebyshev as cb
from oracle import pipeline as pl
from oracle.csr import Csr, chebyshev
from workloads import generator as g

# bounds and width of the 80 000-row workload's float32 form (Lanczos bounds
# of H'), where a fixed 2048-point grid accepted a degree whose true error was
# 6.4 times the threshold
LARGE_BOUNDS = (-2.4635, -0.2951)
LARGE_KT = 0.003


def test_lobatto_evaluation_matches_chebval():
    # the DCT-I evaluation at the Lobatto points against numpy's chebval
    rng = np.random.default_rng(0)
    c = rng.standard_normal(57)
    npts = 300
    x = np.cos(math.pi * np.arange(npts) / (npts - 1))
    ref = npcheb.chebval(x, np.concatenate([[0.5 * c[0]], c[1:]]))
    assert np.max(np.abs(cb.cheb_eval_lobatto(c, npts) - ref)) < 1e-12
    # and against the Eq. 4 recursion the oracle uses elsewhere
    assert np.max(np.abs(cb.cheb_eval(c, x) - ref)) < 1e-12


def test_fit_grid_grows_with_the_degree():
    assert cb.fit_points(8) == 8192 and cb.fit_points(1024) == 8192
    assert cb.fit_points(2048) == 16384 and cb.fit_points(7000) == 56000


def test_degree_meets_tol_fit_on_a_fine_grid():
    # Eq. 7 at the large workload's bounds: the chosen degree's error on a
    # grid 8 times finer than the rule's is below tol_fit, the degree 8 below
    # fails; a fixed 2048-point grid would have accepted a degree whose true
    # error is several times tol_fit
    lo, hi = LARGE_BOUNDS
    tau = 0.5 * (lo + hi)
    f = lambda e: cb.occ_erfc(e, tau, LARGE_KT)
    tol = 1e-6
    m = cb.degree(f, lo, hi, tol, m_start=2048)
    assert cb.fit_error(f, lo, hi, m - 8) >= tol
    assert cb.fit_error(f, lo, hi, m, npts=64 * m) < tol
    assert 2200 <= m <= 2300
    # the old fixed grid: the smallest passing multiple of 8 from 1800 up
    m_old = 1800
    while cb.fit_error(f, lo, hi, m_old, npts=2048) >= tol:
        m_old += 8
    assert m_old < m - 100
    assert cb.fit_error(f, lo, hi, m_old, npts=64 * m_old) > 3 * tol


# ----------------------------------------------------------------------------
# Eq. 6 on designed spectra
# ----------------------------------------------------------------------------

def exact_penalty(lam, lo, hi, alpha=cb.PENALTY_ALPHA):
    """Tr f^p(M~) from the eigenvalues: the value the moment formula
    approximates (f^p is entire, so the expansion also converges just
    outside [-1, 1])."""
    sigma, tau = cb.scale_shift(lo, hi)
    x = sigma * (np.asarray(lam) - tau)
    return float(np.sum(np.exp(alpha * (x + 1.0)) - np.exp(-alpha * (x - 1.0))))


def exact_moments(lam, lo, hi, n):
    """Tr T_k(M~) = sum_i T_k(x_i), T_k(x) = cos(k arccos x) inside [-1, 1]
    and sign(x)^k cosh(k arccosh |x|) outside."""
    sigma, tau = cb.scale_shift(lo, hi)
    x = sigma * (np.asarray(lam) - tau)
    k = np.arange(n)[:, None]
    inside = np.abs(x) <= 1.0
    T = np.where(inside, np.cos(k * np.arccos(np.clip(x, -1, 1))),
                 np.sign(x) ** k * np.cosh(k * np.arccosh(np.maximum(np.abs(x), 1.0))))
    return T.sum(axis=1)


def dense_chain_moments(lam, lo, hi, n, seed=0):
    """Moments of the oracle's chain on V diag(lam) V^T (dense pattern: no
    truncation)."""
    rng = np.random.default_rng(seed)
    nn = len(lam)
    V, _ = np.linalg.qr(rng.standard_normal((nn, nn)))
    M = V @ np.diag(lam) @ V.T
    M = 0.5 * (M + M.T)
    rp = np.arange(0, nn * nn + 1, nn, dtype=np.int64)
    ci = np.tile(np.arange(nn, dtype=np.int32), nn)
    A = Csr(nn, rp, ci, M.ravel().copy())
    K = Csr(nn, rp, ci)
    _, mom = chebyshev(pl.scaled(A, lo, hi), K, n, None)
    return mom


@pytest.mark.parametrize("case", ["inside", "at_lo", "at_hi", "near_inside"])
def test_penalty_from_moments_matches_the_eigenvalues(case):
    # eigenvalues at or just beyond a bound (the growth test cannot see them:
    # T_k stays small over 600 terms): Tr W^p from the moments equals the
    # sum of f^p over the exact eigenvalues, and its sign picks the side
    lo, hi = -1.0, 1.0
    lam = np.linspace(-0.9, 0.9, 24)
    if case == "at_lo":
        lam[0] = lo - 1e-5
    elif case == "at_hi":
        lam[-1] = hi + 1e-5
    elif case == "near_inside":
        lam[0] = lo + 0.002  # inside, but within the penalty's reach
    n = 600
    mom = dense_chain_moments(lam, lo, hi, n)
    assert np.max(np.abs(mom - exact_moments(lam, lo, hi, n))) < 1e-9
    assert cb.growth_ok(mom, len(lam))
    pen = cb.penalty_trace(mom)
    ref = exact_penalty(lam, lo, hi)
    assert abs(pen - ref) <= 1e-9 * max(1.0, abs(ref))
    chk = cb.bounds_check(mom, len(lam))
    assert chk["valid"]
    if case == "inside":
        assert chk["ok"] and abs(pen) < 1e-6
    elif case == "at_hi":
        assert not chk["ok"] and pen < -0.5 and chk["side"] == "hi"
    else:
        assert not chk["ok"] and pen > 0.5 and chk["side"] == "lo"


@pytest.mark.parametrize("case, side", [("far_below", "lo"), ("far_above", "hi")])
def test_growth_failure_takes_the_side_from_the_moments(case, side):
    # an eigenvalue clearly outside: the growth test fails and the moments'
    # sign pattern names the side (the penalty would be rounding noise times
    # cosh(k arccosh|x|) there, so it is not used)
    lam = np.linspace(-0.9, 0.9, 24)
    if case == "far_below":
        lam[0] = -1.02
    else:
        lam[-1] = 1.01
    for n in (40, 600):
        mom = dense_chain_moments(lam, -1.0, 1.0, n)
        assert not cb.growth_ok(mom, 24)
        chk = cb.bounds_check(mom, 24)
        assert not chk["ok"] and chk["side"] == side and math.isnan(chk["penalty"])
        assert cb.moment_side(exact_moments(lam, -1.0, 1.0, n)) == side


def test_short_chain_cannot_use_eq6():
    # with 40 terms the fit of f^p is too poor to trust Eq. 6: an eigenvalue
    # just beyond a bound passes (only the growth test remains)
    lam = np.linspace(-0.9, 0.9, 24)
    lam[0] = -1.0 - 1e-5
    chk = cb.bounds_check(dense_chain_moments(lam, -1.0, 1.0, 40), 24)
    assert not chk["valid"] and math.isnan(chk["penalty"]) and chk["ok"]


def simulate_widening(lam, lo, hi, n_of, max_reexpand=3):
    """The widening rule of reading R7 driven by exact eigenvalues instead of
    chain moments: (final lo, hi, widenings)."""
    n = len(lam)
    r = 0
    while True:
        m = n_of(lo, hi)
        t = exact_moments(lam, lo, hi, m)
        if np.max(np.abs(t)) > 1.01 * n:
            side = cb.moment_side(t)
        else:
            pen = exact_penalty(lam, lo, hi)
            if not (cb.penalty_valid(m, n) and abs(pen) > 0.5):
                return lo, hi, r
            side = "lo" if pen > 0 else "hi"
        assert r < max_reexpand
        w = hi - lo
        if side == "lo":
            lo -= 0.1 * w
        else:
            hi += 0.1 * w
        r += 1


def designed_system(lam, seed=0):
    """H with eigenvalues lam (4 per atom, dense pattern) and S = I."""
    b = 4
    nb = len(lam) // b
    rng = np.random.default_rng(seed)
    V, _ = np.linalg.qr(rng.standard_normal((len(lam), len(lam))))
    Hd = V @ np.diag(lam) @ V.T
    Hd = 0.5 * (Hd + Hd.T)
    rp = np.arange(0, nb * nb + 1, nb, dtype=np.int64)
    ci = np.tile(np.arange(nb, dtype=np.int32), nb)
    pat = g.BlockPattern(nb, b, rp, ci)
    Sv = np.zeros((nb * nb, b, b))
    Sv[np.arange(nb) * nb + np.arange(nb)] = np.eye(b)
    H = pl.BlockMat(nb, b, rp, ci, g.from_dense(pat, Hd))
    S = pl.BlockMat(nb, b, rp, ci, Sv)
    P = pl.BlockMat(nb, b, rp, ci)
    return H, S, P, Hd


@pytest.mark.parametrize("case, expect", [("inside", 0), ("below_015", 2), ("above_005", 1),
                                          ("both", 3), ("at_hi", 1)])
def test_widening_count_and_side_follow_the_exact_eigenvalues(case, expect):
    lo, hi = -1.0, 0.5
    w = hi - lo
    lam = np.linspace(lo + 0.08 * w, hi - 0.08 * w, 24)
    if case == "below_015":
        lam[0] = lo - 0.15 * w
    elif case == "above_005":
        lam[-1] = hi + 0.05 * w
    elif case == "both":
        lam[0] = lo - 0.05 * w
        lam[-1] = hi + 0.12 * w
    elif case == "at_hi":
        lam[-1] = hi + 1e-6
    H, S, P, _ = designed_system(lam)
    kT = 0.02
    n_e = 12.0
    tol = 1e-10
    n_of = lambda a, b_: cb.degree(lambda e: cb.occ_erfc(e, 0.5 * (a + b_), kT), a, b_, tol)
    exp_lo, exp_hi, exp_r = simulate_widening(lam, lo, hi, n_of)
    if expect is not None:
        assert exp_r == expect
    K, info = pl.fermi_operator(H, S, P, n_e, kT, s_bounds_=(0.5, 1.5), n_pl_s=40,
                                h_bounds=(lo, hi), tol_fit=tol)
    assert info["reexpansions"] == exp_r
    assert abs(info["lo"] - exp_lo) < 1e-14 and abs(info["hi"] - exp_hi) < 1e-14
    if case == "below_015":
        assert info["hi"] == hi and info["lo"] < lo
    if case == "above_005":
        assert info["lo"] == lo and info["hi"] > hi
    assert abs(info["penalty"]) < 0.5


def test_widening_gives_the_matrix_function():
    # bounds inside the spectrum on one side: after the widenings the result
    # equals the occupation of the exact eigenvalues (dense pattern, S = I)
    lo, hi = -1.0, 0.5
    w = hi - lo
    lam = np.linspace(lo - 0.15 * w, hi - 0.1 * w, 24)
    H, S, P, Hd = designed_system(lam, seed=3)
    kT, n_e = 0.05, 11.0
    K, info = pl.fermi_operator(H, S, P, n_e, kT, s_bounds_=(0.5, 1.5), n_pl_s=40,
                                h_bounds=(lo, hi), tol_fit=1e-12, tol_fit_s=1e-14)
    assert info["reexpansions"] >= 1
    ev, V = np.linalg.eigh(Hd)
    Kref = V @ np.diag(cb.occ_erfc(ev, info["mu"], kT)) @ V.T
    pat = g.BlockPattern(P.nb, P.b, P.row_ptr, P.col_idx)
    assert np.max(np.abs(g.to_dense(pat, K) - Kref)) < 1e-9
    assert abs(np.sum(cb.occ_erfc(ev, info["mu"], kT)) - n_e) < 1e-6


def simulate_power_widening(lam, lo, hi, n_of, max_reexpand=3):
    """Reading R7 for matrix powers driven by exact eigenvalues: the growth
    test on max(n_pl, penalty_degree(n)) terms (a failure moves both sides by
    10 % of the width), then Eq. 6 from the eigenvalues (a failure moves the
    penalty's side by 2.5 %); the lower bound at most halves.  Returns
    (final lo, hi, widenings)."""
    n = len(lam)
    r = 0
    while True:
        m = max(n_of(lo, hi), cb.penalty_degree(n))
        t = exact_moments(lam, lo, hi, m)
        if np.max(np.abs(t)) > 1.01 * n:
            move_lo = move_hi = True
            step = 0.1
        else:
            pen = exact_penalty(lam, lo, hi)
            if abs(pen) <= 0.5:
                return lo, hi, r
            move_lo, move_hi = pen > 0, pen < 0
            step = 0.025
        assert r < max_reexpand
        w = hi - lo
        if move_lo:
            lo = max(lo - step * w, 0.5 * lo)
        if move_hi:
            hi = hi + step * w
        r += 1


def dense_spd(lam, seed=5):
    """S = V diag(lam) V^T on a dense 4x4-block pattern (no truncation)."""
    nn = len(lam)
    rng = np.random.default_rng(seed)
    V, _ = np.linalg.qr(rng.standard_normal((nn, nn)))
    Sd = V @ np.diag(lam) @ V.T
    Sd = 0.5 * (Sd + Sd.T)
    nb, b = nn // 4, 4
    rp = np.arange(0, nb * nb + 1, nb, dtype=np.int64)
    ci = np.tile(np.arange(nb, dtype=np.int32), nb)
    pat = g.BlockPattern(nb, b, rp, ci)
    S = pl.BlockMat(nb, b, rp, ci, g.from_dense(pat, Sd))
    return S, pl.BlockMat(nb, b, rp, ci), pat, Sd


def test_penalty_degree_makes_eq6_exact_to_its_threshold():
    # with penalty_degree(n) terms, Tr W^p from the moments is within 0.1 of
    # the sum of f^p over the eigenvalues for any spectrum in [-1, 1] (n times
    # the fit error is below 0.1), and with 8 terms fewer it is not trusted
    rng = np.random.default_rng(7)
    for n in (24, 200, 2000):
        m = cb.penalty_degree(n)
        assert m % 8 == 0 and cb.penalty_valid(m, n) and not cb.penalty_valid(m - 8, n)
        lam = np.concatenate([rng.uniform(-1.0, 1.0, n - 2), [-1.0, 0.9995]])
        pen = cb.penalty_trace(exact_moments(lam, -1.0, 1.0, m))
        assert abs(pen - exact_penalty(lam, -1.0, 1.0)) < 0.1
    assert cb.penalty_degree(24) < cb.penalty_degree(2000) <= cb.penalty_degree(10 ** 6) <= 1024


@pytest.mark.parametrize("case, expect", [("inside", 0), ("near_lo", 1), ("near_hi", 1),
                                          ("below", 1), ("far_below", 2)])
@pytest.mark.parametrize("n_pl", [40, None])
def test_matrix_power_bounds_follow_the_exact_eigenvalues(case, expect, n_pl):
    # S^-1 from the bounds [0.5, 2]: an eigenvalue inside but within reach of
    # the penalty (near_lo, near_hi) moves only that side, by 2.5 % of the
    # width; one outside (below) fails the growth test on the check chain and
    # moves both by 10 %; one far below (0.2) needs two widenings, the second
    # halving the lower bound.
    # With 40 terms (fewer than penalty_degree(24) = 48) the bounds are judged
    # on a moments-only chain of 48 terms; with the Eq. 7 degree, on the
    # series' own moments once it reaches 48 terms
    lo, hi = 0.5, 2.0
    w = hi - lo
    lam = np.linspace(lo + 0.08 * w, hi - 0.08 * w, 24)
    if case == "near_lo":
        lam[0] = lo + 0.0005 * w
    elif case == "near_hi":
        lam[-1] = hi - 0.0005 * w
    elif case == "below":
        lam[0] = lo - 0.03 * w
    elif case == "far_below":
        lam[0] = 0.2
    S, P, pat, Sd = dense_spd(lam)
    tol = 1e-12
    n_of = (lambda a, b_: n_pl) if n_pl else (lambda a, b_: cb.degree(cb.power_fn(-1.0), a, b_, tol))
    exp_lo, exp_hi, exp_r = simulate_power_widening(lam, lo, hi, n_of, max_reexpand=6)
    assert exp_r == expect
    val, info = pl.matrix_power(S, -1.0, P, bounds=(lo, hi), n_pl=n_pl, tol_fit=tol, max_reexpand=6)
    assert info["reexpansions"] == exp_r
    assert info["lo"] == exp_lo and info["hi"] == exp_hi
    assert info["check_terms"] == max(info["n_pl"], cb.penalty_degree(24))
    assert abs(info["penalty"]) < 0.5
    if case == "near_lo":
        assert info["lo"] == lo - 0.025 * w and info["hi"] == hi
    if case == "near_hi":
        assert info["lo"] == lo and info["hi"] == hi + 0.025 * w
    if case == "far_below":
        assert info["lo"] == 0.5 * (lo - 0.1 * w)
    if n_pl is None:
        assert np.max(np.abs(g.to_dense(pat, val) - np.linalg.inv(Sd))) < 1e-9


def test_matrix_power_widens_on_growth():
    # S with its smallest eigenvalue far below the guess [0.5, 1]: the growth
    # test fails and both sides widen (the lower one at most halved) until the
    # spectrum is inside; the result is then S^-1 on the dense pattern
    lam = np.linspace(0.2, 1.6, 24)
    S, P, pat, Sd = dense_spd(lam)
    val, info = pl.matrix_power(S, -1.0, P, bounds=(0.5, 1.0), tol_fit=1e-12, max_reexpand=12)
    n_of = lambda a, b_: cb.degree(cb.power_fn(-1.0), a, b_, 1e-12)
    lo, hi, r = simulate_power_widening(lam, 0.5, 1.0, n_of, max_reexpand=12)
    assert info["reexpansions"] == r >= 2
    assert info["lo"] == lo and info["hi"] == hi
    assert np.max(np.abs(g.to_dense(pat, val) - np.linalg.inv(Sd))) < 1e-9


# ----------------------------------------------------------------------------
# truncation order on a sparse pattern
# ----------------------------------------------------------------------------

@pytest.fixture(scope="module")
def sparse_case():
    sysm = g.make_system(60, 4, 4.0, 5.2, seed=11, kT=0.02)
    ph, pk = sysm.pat_h, sysm.pat_k
    assert ph.nnzb < pk.nnzb < ph.nb * ph.nb  # nested and sparse
    H = pl.BlockMat(ph.nb, 4, ph.row_ptr, ph.col_idx, sysm.H)
    S = pl.BlockMat(ph.nb, 4, ph.row_ptr, ph.col_idx, sysm.S)
    P = pl.BlockMat(pk.nb, 4, pk.row_ptr, pk.col_idx)
    X, Hp, _ = pl.orthogonal_frame(H, S, P, s_bnds=(0.25, 2.1), n_pl_s=40)
    mask_h = g.to_dense(ph, np.ones((ph.nnzb, 4, 4)))
    mask_k = g.to_dense(pk, np.ones((pk.nnzb, 4, 4)))
    return dict(sysm=sysm, H=H, S=S, P=P, X=X, Hp=Hp, mask_h=mask_h, mask_k=mask_k)


def test_frame_truncation_order_on_a_sparse_pattern(sparse_case):
    c = sparse_case
    Xd = c["X"].dense()
    Hd = g.to_dense(c["sysm"].pat_h, c["sysm"].H)
    Mh, Mk = c["mask_h"], c["mask_k"]
    Z = Mk * (Hd @ Xd)
    Hp_ref = Mh * (Xd @ Z)
    Hp_ref = 0.5 * (Hp_ref + Hp_ref.T)
    Hp = c["Hp"].dense()
    assert np.max(np.abs(Hp - Hp_ref)) < 1e-13
    assert np.array_equal(Hp, Hp.T)
    assert np.all(Hp[Mh == 0] == 0)
    # truncation matters here: dropping either mask, or swapping them,
    # changes H' by far more than rounding
    assert np.max(np.abs(Mh * (Xd @ (Hd @ Xd)) - Hp_ref)) > 1e-6
    swapped = Mk * (Xd @ (Mh * (Hd @ Xd)))
    assert np.max(np.abs(0.5 * (swapped + swapped.T) - Hp_ref)) > 1e-6


def test_post_transform_truncation_order_on_a_sparse_pattern(sparse_case):
    c = sparse_case
    K = c["P"].pattern_csr()
    rng = np.random.default_rng(12)
    Kp_d = c["mask_k"] * rng.standard_normal(c["mask_k"].shape)
    Kp_d = 0.5 * (Kp_d + Kp_d.T)
    Kp = K.with_values(K.values_from_dense(Kp_d))
    Xd = c["X"].dense()
    Mk = c["mask_k"]
    ref = Mk * (Xd @ (Mk * (Kp_d @ Xd)))
    out = pl.post_transform(Kp, c["X"], K).dense()
    assert np.max(np.abs(out - ref)) < 1e-13
    assert np.max(np.abs(Mk * (Xd @ Kp_d @ Xd) - ref)) > 1e-6


def test_truncated_fermi_operator_and_trace_ks(sparse_case):
    # the whole oracle on the sparse pattern against dense products with
    # explicit masks at the same bounds, degree and mu; Tr(KS) on that
    # truncated K
    c = sparse_case
    sysm = c["sysm"]
    lo, hi = -1.9, 0.2
    n_pl, mu, kT = 300, -0.6, sysm.kT
    Kv, info = pl.fermi_operator(c["H"], c["S"], c["P"], sysm.n_electrons, kT, s_bounds_=(0.25, 2.1),
                                 n_pl_s=40, h_bounds=(lo, hi), n_pl=n_pl, mu=mu)
    Mk = c["mask_k"]
    Hp = c["Hp"].dense()
    sigma, tau = cb.scale_shift(lo, hi)
    Ht = sigma * (Hp - tau * np.eye(Hp.shape[0]))
    coef = cb.cheb_coeffs(lambda e: cb.occ_erfc(e, mu, kT), lo, hi, n_pl)
    T0 = Mk * np.eye(Hp.shape[0])
    T1 = Mk * Ht
    acc = 0.5 * coef[0] * T0 + coef[1] * T1
    for k in range(2, n_pl):
        T0, T1 = T1, Mk * (2.0 * Ht @ T1) - T0
        acc += coef[k] * T1
    Xd = c["X"].dense()
    Kref = Mk * (Xd @ (Mk * (acc @ Xd)))
    Kd = g.to_dense(sysm.pat_k, Kv)
    assert np.max(np.abs(Kd - Kref)) < 1e-11
    Sd = g.to_dense(sysm.pat_h, sysm.S)
    assert abs(info["trKS"] - float(np.sum(Kref * Sd))) < 1e-9
