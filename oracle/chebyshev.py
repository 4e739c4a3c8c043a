"""Oracle, scalar part: Chebyshev coefficients, degree search, occupation
functions, chemical-potential bisection and eigenvalue extraction, in float64.

TEST INFRASTRUCTURE ONLY.  Nothing in the product imports this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark do.  It
shares no code with the HIP path.

Every function is the plain definition from the paper, written for a reader
checking it against the text by eye:

  * Sec. "Expansion in Chebyshev polynomials": the expansion
    p(M) = c_0/2 I + sum_j c_j T_j(M~) (Eq. 1), the scaling
    M~ = sigma (M - tau I) with sigma = 2/(e_max-e_min), tau = (e_min+e_max)/2
    (Eqs. 2-3), the coefficients (Eq. 5).
  * Sec. "Determination of the eigenvalue bounds and polynomial degree": the
    penalty function (Eq. 6) and the degree rule (Eq. 7).
  * Sec. "Fermi Operator Expansion": Fermi function (Eq. 9), the erfc
    occupation (Eq. 11), Tr(KS) = N fixing mu.
  * Sec. "Extraction of selected eigenvalues": the N-th eigenvalue is the mu
    at which the occupation is N - 1/2.

Readings of points the paper leaves open (each is listed in the design notes):
  R1  the sum of Eq. 1 runs over j = 0 .. n_pl-1 (Eq. 5 with n_pl nodes makes
      c_{n_pl} vanish identically);
  R2  Eq. 5's cosine argument is pi*j*(k+1/2)/n_pl;
  R5  erfc occupation f = 1/2 erfc((e - mu)/kT), i.e. beta = 1/kT; Fermi-Dirac
      f = 1/(1 + exp((e - mu)/kT));
  R6  occupations in [0, 1], no spin factor;
  R7  Eq. 6 is evaluated in the scaled variable with the bounds at -1 and 1
      and alpha = -200, so an eigenvalue at a bound contributes 1; the check
      fails when some |Tr T_k| exceeds 1.01 n (growth test; the side then
      comes from the moments' sign pattern), else when |Tr W^p| > 0.5 (only
      when the n-term fit of f^p is good: n times its error, judged on
      min(n, 1024) terms, below 0.1; the sign picks the side); the failing
      side moves out by 10 % of the width;
  R8  Eq. 7's threshold is called tol_fit; the max is taken on
      max(8192, 8 m) Chebyshev-Lobatto points of [lo, hi], a grid that
      grows with m so that the error curve of p_m (about m oscillations) is
      sampled 8 times per oscillation; m runs over 8, 16, 24, ...
  R10 mu by bisection on [lo, hi];
  R12 eigenvalue indices N with N(lo) < N - 1/2 < N(hi), ascending.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special

# ----------------------------------------------------------------------------
# functions that the expansion represents
# ----------------------------------------------------------------------------


def occ_erfc(e, mu: float, kT: float):
    """Eq. 11: f(e) = 1/2 [1 - erf((e - mu)/kT)]."""
    return 0.5 * scipy.special.erfc((np.asarray(e, dtype=np.float64) - mu) / kT)


def occ_fermi_dirac(e, mu: float, kT: float):
    """Eq. 9: f(e) = 1 / (1 + exp((e - mu)/kT)), written with expit for range."""
    return scipy.special.expit(-(np.asarray(e, dtype=np.float64) - mu) / kT)


def power_fn(a: float):
    """Sec. "Matrix powers": f(x) = x^a."""
    return lambda x: np.power(np.asarray(x, dtype=np.float64), a)


def penalty_fn(alpha: float, emin: float, emax: float):
    """Eq. 6: f^p(x) = exp(alpha (x - emin)) - exp(-alpha (x - emax))."""
    def f(x):
        x = np.asarray(x, dtype=np.float64)
        return np.exp(alpha * (x - emin)) - np.exp(-alpha * (x - emax))
    return f


# ----------------------------------------------------------------------------
# Eqs. 2-3 and 5
# ----------------------------------------------------------------------------


def scale_shift(lo: float, hi: float) -> tuple[float, float]:
    """Eq. 3: sigma = 2/(e_max - e_min), tau = (e_min + e_max)/2."""
    return 2.0 / (hi - lo), 0.5 * (lo + hi)


def cheb_coeffs(f, lo: float, hi: float, n_pl: int) -> np.ndarray:
    """Eq. 5 as printed (readings R1, R2):

    c_j = 2/n sum_{k=0}^{n-1} f(cos(pi (k+1/2)/n)/sigma + tau) cos(pi j (k+1/2)/n),
    for j = 0 .. n-1.
    """
    sigma, tau = scale_shift(lo, hi)
    k = np.arange(n_pl, dtype=np.float64)
    theta = math.pi * (k + 0.5) / n_pl
    fx = f(np.cos(theta) / sigma + tau)
    c = np.empty(n_pl)
    # c_j = 2/n sum_k fx_k cos(j theta_k), in row chunks to bound memory
    for j0 in range(0, n_pl, 256):
        j = np.arange(j0, min(j0 + 256, n_pl), dtype=np.float64)
        c[j0:j0 + j.shape[0]] = 2.0 / n_pl * (np.cos(np.outer(j, theta)) @ fx)
    return c


def cheb_eval(c: np.ndarray, xs: np.ndarray) -> np.ndarray:
    """Eq. 1 for scalars: c_0/2 + sum_{j>=1} c_j T_j(xs), T by the Eq. 4 recursion."""
    xs = np.asarray(xs, dtype=np.float64)
    t_prev = np.ones_like(xs)
    out = 0.5 * c[0] * t_prev
    if c.shape[0] == 1:
        return out
    t = xs.copy()
    out = out + c[1] * t
    for j in range(2, c.shape[0]):
        t_next = 2.0 * xs * t - t_prev
        out = out + c[j] * t_next
        t_prev, t = t, t_next
    return out


def lobatto_grid(lo: float, hi: float, npts: int = 8192) -> np.ndarray:
    """Chebyshev-Lobatto points of [lo, hi] (reading R8)."""
    sigma, tau = scale_shift(lo, hi)
    return np.cos(math.pi * np.arange(npts) / (npts - 1)) / sigma + tau


def fit_points(m: int) -> int:
    """Reading R8: number of Lobatto points on which Eq. 7's max is taken."""
    return max(8192, 8 * m)


def cheb_eval_lobatto(c: np.ndarray, npts: int) -> np.ndarray:
    """Eq. 1 for scalars at the Lobatto points x_i = cos(pi i/(npts-1)):
    c_0/2 + sum_j c_j cos(pi i j/(npts-1)), which is a DCT-I (library
    routine) of (c_0/2, c_1/2, ..., c_{m-1}/2, 0, ..., 0)."""
    import scipy.fft
    assert npts - 1 >= c.shape[0]
    a = np.zeros(npts)
    a[:c.shape[0]] = 0.5 * c
    a[0] = 0.5 * c[0]
    # scipy's DCT-I: y_i = a_0 + (-1)^i a_{N-1} + 2 sum_{j=1}^{N-2} a_j cos(pi i j/(N-1))
    return scipy.fft.dct(a, type=1)


def fit_error(f, lo: float, hi: float, m: int, npts: int | None = None) -> float:
    """Eq. 7's max |p_m - f| over the Lobatto grid of reading R8 (npts points,
    default fit_points(m)); p_m is the Eq. 5 interpolant with m terms."""
    npts = fit_points(m) if npts is None else npts
    x = lobatto_grid(lo, hi, npts)
    c = cheb_coeffs(f, lo, hi, m)
    if npts - 1 >= m:
        p = cheb_eval_lobatto(c, npts)
    else:  # a grid coarser than the expansion (only to show what it misses)
        sigma, tau = scale_shift(lo, hi)
        p = cheb_eval(c, sigma * (x - tau))
    return float(np.max(np.abs(p - f(x))))


def degree(f, lo: float, hi: float, tol_fit: float, step: int = 8,
           m_max: int = 4000, npts: int | None = None, m_start: int | None = None) -> int:
    """Eq. 7: the smallest m (m = step, 2 step, ...) with max|p_m - f| < tol_fit.

    m_start (a multiple of step) starts the scan later; it is only for
    callers that already know every smaller m fails."""
    m = step if m_start is None else m_start
    while m <= m_max:
        if fit_error(f, lo, hi, m, npts) < tol_fit:
            return m
        m += step
    raise ValueError("no degree up to m_max meets tol_fit")


# ----------------------------------------------------------------------------
# Eq. 6: the check of the spectral bounds (reading R7)
# ----------------------------------------------------------------------------

PENALTY_ALPHA = -200.0


def penalty_trace(t: np.ndarray, alpha: float = PENALTY_ALPHA) -> float:
    """Tr W^p of Eq. 6 from the moments t_k = Tr T_k(M~) of the scaled matrix:
    W^p = c_0/2 I + sum_j c_j T_j(M~) with c the Eq. 5 coefficients of
    f^p(x) = exp(alpha (x + 1)) - exp(-alpha (x - 1)) on [-1, 1], as many as
    there are moments."""
    t = np.asarray(t, dtype=np.float64)
    c = cheb_coeffs(penalty_fn(alpha, -1.0, 1.0), -1.0, 1.0, t.shape[0])
    return trace_from_moments(c, t)


def penalty_valid(n_terms: int, n_rows: int, alpha: float = PENALTY_ALPHA) -> bool:
    """Reading R7: Eq. 6 is trusted only when n_rows times the fit error of
    f^p (with min(n_terms, 1024) terms) is below 0.1."""
    m = min(n_terms, 1024)
    return fit_error(penalty_fn(alpha, -1.0, 1.0), -1.0, 1.0, m) * n_rows < 0.1


def penalty_degree(n_rows: int, step: int = 8) -> int:
    """Reading R7 for matrix powers: the fewest terms (a multiple of step, at
    most 1024) with which Eq. 6 is trusted on n_rows rows (penalty_valid).
    A power series shorter than this is checked on a moments-only chain of
    this many terms before it is accumulated."""
    m = step
    while m < 1024 and not penalty_valid(m, n_rows):
        m += step
    return m


def growth_ok(t: np.ndarray, n_rows: int) -> bool:
    """|T_k(x)| <= 1 on [-1, 1], so |Tr T_k| <= n whenever every eigenvalue of
    M~ is inside the bounds; reading R7 allows 1 %."""
    t = np.asarray(t, dtype=np.float64)
    return bool(np.all(np.isfinite(t)) and np.all(np.abs(t) <= 1.01 * n_rows))


def moment_side(t: np.ndarray) -> str:
    """Side of an eigenvalue far outside the bounds, from the moments alone:
    for x < -1, T_k(x) = (-1)^k cosh(k arccosh|x|) alternates in sign, for
    x > 1 it keeps one sign, and it grows fastest at the largest k.  Over the
    last 16 moments, 'lo' when the alternating sum is the larger one."""
    t = np.asarray(t, dtype=np.float64)
    k = np.arange(max(0, t.shape[0] - 16), t.shape[0])
    tt = np.nan_to_num(t[k], nan=0.0, posinf=1e300, neginf=-1e300)
    alt = abs(float(np.sum(np.where(k % 2 == 0, tt, -tt))))
    same = abs(float(np.sum(tt)))
    return "lo" if alt > same else "hi"


def bounds_check(t: np.ndarray, n_rows: int) -> dict:
    """Eq. 6 and the growth test on the moments of one chain (reading R7).

    The growth test comes first: an eigenvalue clearly outside the bounds
    makes some |Tr T_k| exceed 1.01 n, and then the rounding noise of the
    penalty coefficients times that growth decides the penalty's value, so
    the side comes from the moments' sign pattern (moment_side).  With the
    growth test passed, Eq. 6 (when its fit is valid) catches eigenvalues at
    or just beyond a bound and its sign picks the side: positive for the
    lower bound, negative for the upper one.

    Returns ok, the penalty (NaN when not evaluated) and, when not ok, the
    side to move: 'lo' or 'hi'."""
    if not growth_ok(t, n_rows):
        return dict(ok=False, penalty=math.nan, valid=False, side=moment_side(t))
    valid = penalty_valid(len(t), n_rows)
    pen = penalty_trace(t) if valid else math.nan
    ok = not (valid and abs(pen) > 0.5)
    side = None if ok else ("lo" if pen > 0 else "hi")
    return dict(ok=ok, penalty=pen, valid=valid, side=side)


def widen(lo: float, hi: float, side: str) -> tuple[float, float]:
    """Reading R7: move the failing side out by 10 % of the width."""
    w = hi - lo
    if side in ("lo", "both"):
        lo -= 0.1 * w
    if side in ("hi", "both"):
        hi += 0.1 * w
    return lo, hi


# ----------------------------------------------------------------------------
# trace-moment formulas (Eq. 1 taken under the trace)
# ----------------------------------------------------------------------------


def trace_from_moments(c: np.ndarray, t: np.ndarray) -> float:
    """Tr p(M~) = c_0/2 Tr T_0 + sum_{j>=1} c_j Tr T_j, with t_j = Tr T_j."""
    return float(0.5 * c[0] * t[0] + np.dot(c[1:], t[1:c.shape[0]]))


def energy_traces(t: np.ndarray, lo: float, hi: float) -> np.ndarray:
    """Tr(T_k H') for k = 0 .. len(t) - 2 from the moments t_k = Tr T_k(H~).

    Sec. "Fermi Operator Expansion" checks the width of the occupation with
    the energy E = Tr(K H) (= Tr(K' H') in the orthogonal frame).  With
    H~ = sigma (H' - tau I) (Eqs. 2-3), H' = H~/sigma + tau I, and
    Tr(T_k H~) follows from the recursion 2 x T_k = T_{k+1} + T_{k-1}:
    Tr(T_0 H~) = t_1 and Tr(T_k H~) = (t_{k+1} + t_{k-1}) / 2 for k >= 1.
    The truncated recursion keeps every diagonal block (the diagonal is in
    P_K), so these traces are exact for the truncated chain too."""
    sigma, tau = scale_shift(lo, hi)
    t = np.asarray(t, dtype=np.float64)
    m = t.shape[0] - 1
    g = np.empty(m)
    g[0] = t[1]
    g[1:] = 0.5 * (t[2:m + 1] + t[0:m - 1])
    return g / sigma + tau * t[:m]


def energy_from_moments(c: np.ndarray, t: np.ndarray, lo: float, hi: float) -> float:
    """E = Tr(p(H') H') = c_0/2 Tr(T_0 H') + sum_j c_j Tr(T_j H') (Eq. 1);
    needs one moment more than coefficients."""
    e = energy_traces(t, lo, hi)
    n = c.shape[0]
    assert e.shape[0] >= n
    return float(0.5 * c[0] * e[0] + np.dot(c[1:], e[1:n]))


def electron_count(mu: float, t: np.ndarray, lo: float, hi: float, kT: float,
                   smearing: str = "erfc") -> float:
    """Tr K'(mu) in the orthogonal frame = N(mu), from the moments of H~'."""
    occ = occ_erfc if smearing == "erfc" else occ_fermi_dirac
    c = cheb_coeffs(lambda e: occ(e, mu, kT), lo, hi, t.shape[0])
    return trace_from_moments(c, t)


def bisect_mu(t: np.ndarray, lo: float, hi: float, kT: float, n_target: float,
              tol_n: float, smearing: str = "erfc", mu_lo: float | None = None,
              mu_hi: float | None = None, max_iter: int = 200) -> tuple[float, int]:
    """Reading R10: bisection for N(mu) = n_target on [mu_lo, mu_hi].

    N(mu) increases with mu.  Stops when |N - n_target| <= tol_n or the bracket
    is below 1e-13; returns (mu, iterations)."""
    a = lo if mu_lo is None else mu_lo
    b = hi if mu_hi is None else mu_hi
    it = 0
    mid = 0.5 * (a + b)
    while it < max_iter:
        it += 1
        mid = 0.5 * (a + b)
        nm = electron_count(mid, t, lo, hi, kT, smearing)
        if abs(nm - n_target) <= tol_n or (b - a) <= 1e-13:
            break
        if nm < n_target:
            a = mid
        else:
            b = mid
    return mid, it


def eigenvalues_from_moments(t: np.ndarray, lo: float, hi: float, kT: float,
                             e_lo: float, e_hi: float, smearing: str = "erfc",
                             tol_e: float = 1e-12) -> np.ndarray:
    """Sec. "Extraction of selected eigenvalues" (reading R12): for every N with
    N(e_lo) < N - 1/2 < N(e_hi), the mu solving N(mu) = N - 1/2 by bisection."""
    n_lo = electron_count(e_lo, t, lo, hi, kT, smearing)
    n_hi = electron_count(e_hi, t, lo, hi, kT, smearing)
    first = int(math.floor(n_lo + 0.5)) + 1
    last = int(math.floor(n_hi + 0.5))
    out = []
    for N in range(first, last + 1):
        target = N - 0.5
        if not (n_lo < target < n_hi):
            continue
        a, b = e_lo, e_hi
        while b - a > tol_e:
            mid = 0.5 * (a + b)
            if electron_count(mid, t, lo, hi, kT, smearing) < target:
                a = mid
            else:
                b = mid
        out.append(0.5 * (a + b))
    return np.asarray(out)


def homo_lumo_from_moments(t: np.ndarray, lo: float, hi: float, kT: float, n_e: float,
                           smearing: str = "erfc", tol_n: float | None = None) -> tuple[float, float]:
    """Sec. "Extraction of selected eigenvalues" (reading R19): the moments of
    a density-kernel chain give rough HOMO and LUMO estimates.  With
    N_h = ceil(N_e) occupied states, eigenvalue N_h solves N(e) = N_h - 1/2
    and eigenvalue N_h + 1 solves N(e) = N_h + 1/2, at the chain's own width
    kT, bisected on [lo - 20 kT, hi + 20 kT].  NaN where the index is outside
    1..n (n = t_0 = Tr T_0)."""
    n = int(round(t[0]))
    nh = math.ceil(n_e - 1e-9)
    tol = 1e-10 * max(1.0, n_e) if tol_n is None else tol_n
    a, b = lo - 20 * kT, hi + 20 * kT
    homo = bisect_mu(t, lo, hi, kT, nh - 0.5, tol, smearing, a, b)[0] if nh >= 1 else math.nan
    lumo = bisect_mu(t, lo, hi, kT, nh + 0.5, tol, smearing, a, b)[0] if nh + 1 <= n else math.nan
    return homo, lumo


# ----------------------------------------------------------------------------
# spectral bounds (the plain estimates the method starts from)
# ----------------------------------------------------------------------------


def gershgorin(A: np.ndarray | "scipy.sparse.spmatrix") -> tuple[float, float]:
    """[min_i (a_ii - R_i), max_i (a_ii + R_i)], R_i = sum_{j != i} |a_ij|."""
    import scipy.sparse as sp
    if sp.issparse(A):
        A = A.tocsr()
        d = A.diagonal()
        r = np.asarray(abs(A).sum(axis=1)).ravel() - np.abs(d)
    else:
        d = np.diag(A)
        r = np.abs(A).sum(axis=1) - np.abs(d)
    return float(np.min(d - r)), float(np.max(d + r))


def lanczos_extremes(matvec, n: int, k: int, seed: int = 0) -> tuple[float, float, float, float]:
    """k steps of Lanczos with full reorthogonalisation from a seeded start.

    Returns (theta_min, theta_max, res_min, res_max): the extreme Ritz values
    and their residual norms |beta_k s_k|."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n)
    v /= np.linalg.norm(v)
    V = np.zeros((k + 1, n))
    V[0] = v
    alpha = np.zeros(k)
    beta = np.zeros(k)
    m = k
    for j in range(k):
        w = matvec(V[j])
        alpha[j] = np.dot(V[j], w)
        w = w - V[: j + 1].T @ (V[: j + 1] @ w)
        w = w - V[: j + 1].T @ (V[: j + 1] @ w)
        beta[j] = np.linalg.norm(w)
        if beta[j] < 1e-14:
            m = j + 1
            break
        V[j + 1] = w / beta[j]
    T = np.diag(alpha[:m]) + np.diag(beta[: m - 1], 1) + np.diag(beta[: m - 1], -1)
    th, s = np.linalg.eigh(T)
    res = np.abs(beta[m - 1] * s[-1, :])
    return float(th[0]), float(th[-1]), float(res[0]), float(res[-1])
