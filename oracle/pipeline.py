"""Oracle, the method step by step (plain CPU, float64): Fermi-operator
expansion, matrix powers and eigenvalues in an interval, on fixed patterns.

TEST INFRASTRUCTURE ONLY.  Steps follow the paper in its order:

 1. bounds of S (given, or Gershgorin's upper bound and a Lanczos lower bound);
 2. X = S^{-1/2} by the truncated chain on S~ = sigma_S (S - tau_S I)
    (Sec. "Matrix powers": the FOE machinery with f(x) = x^a);
 3. H' = P_H o (X P_K o (H X)), then symmetrised (Sec. "Fermi Operator
    Expansion": the input is replaced by S^-1/2 H S^-1/2; reading R3 applies
    the scale and shift in that orthogonal frame, reading R4 keeps H' on the
    pattern of H, the "sparser Hamiltonian" of Sec. "Fixed versus variable
    sparsity");
 4. bounds of H' (given, or Gershgorin), sigma and tau by Eq. 3;
 5. n_pl by Eq. 7 at mu = tau (given values skip this);
 6. the chain on H~' with the moments t_k = Tr T_k;
 7. mu by bisection on N(mu) = sum' c_k(mu) t_k (= Tr K'(mu) by linearity of
    Eq. 1; reading R9), unless mu is given;
 8. K' = sum' c_k(mu) T_k by a second pass of the chain;
 9. K = P_K o (X P_K o (K' X)), the post-processing S^-1/2 p S^-1/2.

Every value array is in block-CSR order [nnzb, b, b] at the interface and is
converted to scalar CSR inside; the chain itself is csr_chain.c.
"""
from __future__ import annotations

import numpy as np

from . import chebyshev as cb
from .csr import (Csr, block_pattern_to_csr, block_values_to_csr, chebyshev,
                  csr_values_to_block, masked_spgemm)


class BlockMat:
    """A block-CSR matrix given to the oracle: pattern + [nnzb, b, b] values."""

    def __init__(self, nb, b, row_ptr, col_idx, val=None):
        self.nb, self.b = int(nb), int(b)
        self.row_ptr = np.asarray(row_ptr, dtype=np.int64)
        self.col_idx = np.asarray(col_idx, dtype=np.int32)
        self.val = None if val is None else np.asarray(val, dtype=np.float64).reshape(-1, b, b)
        self._csr = None

    def csr(self) -> Csr:
        if self._csr is None:
            self._csr = block_pattern_to_csr(self.nb, self.b, self.row_ptr, self.col_idx)
        c = Csr(self._csr.n, self._csr.rp, self._csr.ci)
        if self.val is not None:
            c.v = block_values_to_csr(self.nb, self.b, self.row_ptr, self.val)
        return c

    def pattern_csr(self) -> Csr:
        if self._csr is None:
            self._csr = block_pattern_to_csr(self.nb, self.b, self.row_ptr, self.col_idx)
        return self._csr

    def to_block(self, v_csr) -> np.ndarray:
        return csr_values_to_block(self.nb, self.b, self.row_ptr, v_csr)


def scaled(A: Csr, lo: float, hi: float) -> Csr:
    """Eq. 2: sigma (A - tau I) with sigma, tau from Eq. 3."""
    sigma, tau = cb.scale_shift(lo, hi)
    r = np.repeat(np.arange(A.n), np.diff(A.rp))
    v = A.v.copy()
    v[r == A.ci] -= tau
    return A.with_values(sigma * v)


def symmetrised(A: Csr) -> Csr:
    M = A.to_scipy()
    Ms = (M + M.T) * 0.5
    return A.with_values(np.asarray(Ms[np.repeat(np.arange(A.n), np.diff(A.rp)), A.ci]).ravel())


def transpose_on(A: Csr) -> Csr:
    """A^T on the same (symmetric) pattern."""
    M = A.to_scipy().T.tocsr()
    return A.with_values(np.asarray(M[np.repeat(np.arange(A.n), np.diff(A.rp)), A.ci]).ravel())


def s_bounds(S: Csr, lanczos_k: int = 60, margin: float = 1e-3) -> tuple[float, float]:
    """Upper: Gershgorin.  Lower: Gershgorin if positive, else the smallest
    Lanczos Ritz value minus its residual and a relative margin."""
    glo, ghi = cb.gershgorin(S.to_scipy())
    if glo > 0:
        return glo, ghi
    M = S.to_scipy()
    tmin, tmax, rmin, rmax = cb.lanczos_extremes(lambda x: M @ x, S.n, min(lanczos_k, S.n))
    lo = tmin - rmin - margin * (ghi - tmin)
    if lo <= 0:
        raise ValueError("S is not positive definite to within the Lanczos estimate")
    return lo, ghi


def widen_power(lo: float, hi: float, side: str = "both") -> tuple[float, float]:
    """Reading R7 for matrix powers.  After a failed growth test ('both': an
    eigenvalue clearly outside, and the bounds may be off on both sides, as
    for a default guess) both sides move out by 10 % of the width.  After a
    failed Eq. 6 ('lo' or 'hi': an eigenvalue at or within about 1 % of that
    bound) only that side moves, by 2.5 % of the width: x^a is steepest at
    the lower bound, where a larger step costs terms and precision.  The
    lower bound at most halves, so that it stays positive for non-integer or
    negative exponents."""
    w = hi - lo
    step = 0.1 if side == "both" else 0.025
    if side in ("lo", "both"):
        lo = max(lo - step * w, 0.5 * lo)
    if side in ("hi", "both"):
        hi = hi + step * w
    return lo, hi


def matrix_power(S: BlockMat, a: float, pattern: BlockMat, bounds=None, n_pl=None,
                 tol_fit: float = 1e-12, extra_powers=(), max_reexpand: int = 3):
    """Sec. "Matrix powers": S^a on `pattern` by the chain with f = x^a.
    Returns (values [nnzb, b, b], info) (and extra powers from the same chain
    when `extra_powers` is given: a dict a' -> values).

    Sec. "Determination of the eigenvalue bounds and polynomial degree": the
    bounds are judged by the growth test and Eq. 6 (reading R7) on the
    moments of at least penalty_degree(n) terms.  A shorter series is first
    checked on a moments-only chain of that length; a longer one is checked
    on its own moments.  A failure widens the bounds (widen_power: both sides
    by 10 % of the width after the growth test, the penalty's side by 2.5 %
    after Eq. 6) and redoes the
    check, at most max_reexpand times; info['reexpansions'] counts the
    widenings, info['penalty'] is Tr W^p for the final bounds and
    info['check_terms'] the number of moments it was judged on."""
    Sc = S.csr()
    K = pattern.pattern_csr()
    lo, hi = bounds if bounds is not None else s_bounds(Sc)
    powers = (a,) + tuple(extra_powers)
    n_given = n_pl
    n_check = cb.penalty_degree(K.n)
    reexp = 0
    while True:
        if n_given is None:
            n_pl = max(cb.degree(cb.power_fn(p), lo, hi, tol_fit) for p in powers)
        St = scaled(Sc, lo, hi)
        if n_pl < n_check:
            # too few terms for Eq. 6: judge the bounds on a moments-only
            # chain of n_check terms before accumulating
            _, mom_chk = chebyshev(St, K, n_check, None)
            chk = cb.bounds_check(mom_chk, K.n)
        if n_pl >= n_check or chk["ok"]:
            coefs = np.stack([cb.cheb_coeffs(cb.power_fn(p), lo, hi, n_pl) for p in powers])
            acc, mom = chebyshev(St, K, n_pl, coefs)
            if n_pl >= n_check:
                chk = cb.bounds_check(mom, K.n)
        if chk["ok"]:
            break
        if reexp >= max_reexpand:
            raise ValueError(f"bounds [{lo}, {hi}] still fail after {reexp} widenings")
        lo, hi = widen_power(lo, hi, chk["side"] if chk["valid"] else "both")
        reexp += 1
    # left-multiplication chain -> values are those of p(S~) directly
    outs = [pattern.to_block(acc[q]) for q in range(len(powers))]
    info = dict(lo=lo, hi=hi, n_pl=n_pl, moments=mom, reexpansions=reexp,
                penalty=chk["penalty"], check_terms=max(n_pl, n_check))
    if extra_powers:
        return outs[0], info, {p: o for p, o in zip(extra_powers, outs[1:])}
    return outs[0], info


def frame_products(H: Csr, X: Csr, K: Csr) -> Csr:
    """Step 3: H' = P_H o (X P_K o (H X)) (reading R4: the inner product on
    the kernel pattern, the outer one on the pattern of H), symmetrised."""
    Z = K.with_values(masked_spgemm(H, X, K))           # P_K o (H X)
    Hp = H.with_values(masked_spgemm(X, Z, H))          # P_H o (X Z)
    return symmetrised(Hp)


def post_transform(Kp: Csr, X: Csr, K: Csr) -> Csr:
    """Step 9: K = P_K o (X P_K o (K' X)), both products on the kernel
    pattern (the post-processing S^-1/2 p S^-1/2 of Sec. "Fermi Operator
    Expansion")."""
    W = K.with_values(masked_spgemm(Kp, X, K))          # P_K o (K' X)
    return K.with_values(masked_spgemm(X, W, K))         # P_K o (X W)


def orthogonal_frame(H: BlockMat, S: BlockMat, pattern: BlockMat, s_bnds=None, n_pl_s=None,
                     tol_fit_s: float = 1e-12):
    """Steps 1-3: returns (X on P_K as Csr, H' on P_H as Csr, info)."""
    Xv, sinfo = matrix_power(S, -0.5, pattern, bounds=s_bnds, n_pl=n_pl_s, tol_fit=tol_fit_s)
    K = pattern.pattern_csr()
    X = K.with_values(block_values_to_csr(pattern.nb, pattern.b, pattern.row_ptr, Xv))
    return X, frame_products(H.csr(), X, K), sinfo


def fermi_operator(H: BlockMat, S: BlockMat, pattern: BlockMat, n_e: float, kT: float,
                   smearing: str = "erfc", s_bounds_=None, n_pl_s=None, h_bounds=None,
                   n_pl=None, mu=None, tol_fit: float = 1e-12, tol_fit_s: float = 1e-12,
                   tol_ne: float | None = None, adapt_kt: bool = False, kt_ratio: float = 1.25,
                   tol_energy: float | None = None, max_kt_halvings: int = 4,
                   max_reexpand: int = 3):
    """Steps 1-9.  Returns (K values [nnzb_K, b, b], info dict).

    adapt_kt: the width check of Sec. "Fermi Operator Expansion": after mu is
    found for kT, a second occupation of width kT' = kt_ratio kT (its own mu
    for the same N) gives E'; if |E - E'| > tol_energy the width is halved and
    the expansion redone (a new degree unless n_pl is given), at most
    max_kt_halvings times.  E and E' come from the moments of the same chain
    (energy_from_moments), which runs one term longer for that.

    The bounds of H' (given or Gershgorin) are checked by Eq. 6 and the
    growth test on the moments of each chain (reading R7); a failure moves
    the failing side out by 10 % of the width and redoes the expansion, at
    most max_reexpand times (info['reexpansions'], info['penalty'])."""
    X, Hp, sinfo = orthogonal_frame(H, S, pattern, s_bounds_, n_pl_s, tol_fit_s)
    K = pattern.pattern_csr()
    lo, hi = h_bounds if h_bounds is not None else cb.gershgorin(Hp.to_scipy())
    sigma, tau = cb.scale_shift(lo, hi)
    occ = cb.occ_erfc if smearing == "erfc" else cb.occ_fermi_dirac
    Ht = scaled(Hp, lo, hi)
    tol_ne = 1e-8 * n_e if tol_ne is None else tol_ne
    tol_e = 1e-4 * n_e if tol_energy is None else tol_energy
    n_pl_given = n_pl
    halvings = 0
    energy = energy_wide = float("nan")
    reexp = 0
    penalty = float("nan")
    while True:
        # step 5-6, checked by Eq. 6 and the growth test (reading R7): the
        # failing side moves out and the expansion is redone
        while True:
            sigma, tau = cb.scale_shift(lo, hi)
            Ht = scaled(Hp, lo, hi)
            n_pl = n_pl_given if n_pl_given is not None else cb.degree(lambda e: occ(e, tau, kT), lo, hi, tol_fit)
            _, mom_e = chebyshev(Ht, K, n_pl + 1 if adapt_kt else n_pl, None)
            chk = cb.bounds_check(mom_e, K.n)
            penalty = chk["penalty"]
            if chk["ok"]:
                break
            if reexp >= max_reexpand:
                raise ValueError(f"bounds [{lo}, {hi}] still fail after {reexp} widenings")
            lo, hi = cb.widen(lo, hi, chk["side"])
            reexp += 1
        mom = mom_e[:n_pl]
        it = 0
        mu_k = mu
        if mu_k is None:
            mu_k, it = cb.bisect_mu(mom, lo, hi, kT, n_e, tol_ne, smearing)
        if not adapt_kt:
            break
        c = cb.cheb_coeffs(lambda e: occ(e, mu_k, kT), lo, hi, n_pl)
        energy = cb.energy_from_moments(c, mom_e, lo, hi)
        kT2 = kt_ratio * kT
        mu2, _ = cb.bisect_mu(mom, lo, hi, kT2, n_e, tol_ne, smearing)
        c2 = cb.cheb_coeffs(lambda e: occ(e, mu2, kT2), lo, hi, n_pl)
        energy_wide = cb.energy_from_moments(c2, mom_e, lo, hi)
        if abs(energy - energy_wide) <= tol_e or halvings >= max_kt_halvings:
            break
        kT *= 0.5
        halvings += 1
    mu = mu_k
    homo, lumo = cb.homo_lumo_from_moments(mom, lo, hi, kT, n_e, smearing)
    c = cb.cheb_coeffs(lambda e: occ(e, mu, kT), lo, hi, n_pl)
    acc, _ = chebyshev(Ht, K, n_pl, c[None, :])
    Kfin = post_transform(K.with_values(acc[0]), X, K)
    Kv = Kfin.v
    Sc = S.csr()
    trKS = float(Kfin.to_scipy().multiply(Sc.to_scipy()).sum())
    info = dict(mu=mu, lo=lo, hi=hi, n_pl=n_pl, n_pl_s=sinfo["n_pl"], s_lo=sinfo["lo"],
                s_hi=sinfo["hi"], moments=mom, bisect_iters=it, trKS=trKS,
                ne_chain=cb.trace_from_moments(c, mom), energy=energy,
                energy_wide=energy_wide, kT=kT, kt_halvings=halvings, homo=homo, lumo=lumo,
                reexpansions=reexp, penalty=penalty)
    return pattern.to_block(Kv), info


def eigs_in_interval(H: BlockMat, S: BlockMat, pattern: BlockMat, e_lo: float, e_hi: float,
                     width: float = 1e-3, s_bounds_=None, n_pl_s=None, h_bounds=None,
                     n_pl=None, tol_fit: float = 1e-6, smearing: str = "erfc"):
    """Sec. "Extraction of selected eigenvalues": chain moments on H~', then the
    mu at which the occupation is N - 1/2 for each N inside [e_lo, e_hi]."""
    X, Hp, sinfo = orthogonal_frame(H, S, pattern, s_bounds_, n_pl_s)
    K = pattern.pattern_csr()
    lo, hi = h_bounds if h_bounds is not None else cb.gershgorin(Hp.to_scipy())
    sigma, tau = cb.scale_shift(lo, hi)
    occ = cb.occ_erfc if smearing == "erfc" else cb.occ_fermi_dirac
    if n_pl is None:
        n_pl = cb.degree(lambda e: occ(e, tau, width), lo, hi, tol_fit)
    _, mom = chebyshev(scaled(Hp, lo, hi), K, n_pl, None)
    ev = cb.eigenvalues_from_moments(mom, lo, hi, width, e_lo, e_hi, smearing)
    return ev, dict(lo=lo, hi=hi, n_pl=n_pl, moments=mom)
