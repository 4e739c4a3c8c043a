"""Oracle, dense definitions (float64, LAPACK through SciPy).

TEST INFRASTRUCTURE ONLY.

These are the exact results the method approximates, written from their
definitions rather than from the method's steps:

  * density kernel, Sec. "Fermi Operator Expansion": solve H c_i = e_i S c_i
    with c_i^T S c_i = 1; K_ab = sum_i f(e_i) c_ia c_ib (Eq. 10) with f the
    occupation of Eq. 11 (or Eq. 9) and mu fixed by sum_i f(e_i) = N, which is
    Tr(KS) = N;
  * matrix powers, Sec. "Comparison with other methods": M = U D U^T,
    M^a = U D^a U^T (the paper's own diagonalisation route);
  * selected eigenvalues: the generalized eigenvalues in [lo, hi];
  * the error measures of Eqs. 12 and 13 (and the relative variant used for
    the inverse accuracy test, which only counts |ref| > 1e-12).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .chebyshev import occ_erfc, occ_fermi_dirac


def generalized_eigh(Hd: np.ndarray, Sd: np.ndarray):
    e, C = scipy.linalg.eigh(Hd, Sd)
    return e, C


def mu_exact(e: np.ndarray, n_e: float, kT: float, smearing: str = "erfc",
             tol: float = 1e-14) -> float:
    occ = occ_erfc if smearing == "erfc" else occ_fermi_dirac
    a, b = float(e[0]) - 50 * kT - 1.0, float(e[-1]) + 50 * kT + 1.0
    while b - a > tol * max(1.0, abs(a) + abs(b)):
        mid = 0.5 * (a + b)
        if np.sum(occ(e, mid, kT)) < n_e:
            a = mid
        else:
            b = mid
    return 0.5 * (a + b)


def density_kernel(Hd: np.ndarray, Sd: np.ndarray, n_e: float, kT: float,
                   smearing: str = "erfc", mu: float | None = None):
    """Returns (K dense, mu, eigenvalues)."""
    e, C = generalized_eigh(Hd, Sd)
    if mu is None:
        mu = mu_exact(e, n_e, kT, smearing)
    occ = occ_erfc if smearing == "erfc" else occ_fermi_dirac
    f = occ(e, mu, kT)
    K = (C * f[None, :]) @ C.T
    return K, mu, e


def matrix_power(Md: np.ndarray, a: float) -> np.ndarray:
    d, U = np.linalg.eigh(Md)
    if np.any(d <= 0) and a != int(a):
        raise ValueError("non-integer power of a matrix that is not positive definite")
    return (U * np.power(d, a)[None, :]) @ U.T


def eigenvalues_in(Hd: np.ndarray, Sd: np.ndarray, lo: float, hi: float) -> np.ndarray:
    e = scipy.linalg.eigh(Hd, Sd, eigvals_only=True)
    return e[(e >= lo) & (e <= hi)]


def w_sparse(f_hat: np.ndarray, f_ref: np.ndarray, relative: bool = False) -> float:
    """Eq. 13 over the entries of the pattern of f_hat (both given as the
    pattern's value arrays)."""
    f_hat = np.asarray(f_hat).ravel()
    f_ref = np.asarray(f_ref).ravel()
    if relative:
        keep = np.abs(f_ref) > 1e-12
        d = (f_hat[keep] - f_ref[keep]) / f_ref[keep]
    else:
        d = f_hat - f_ref
    return float(np.sqrt(np.sum(d * d)) / f_hat.shape[0])


def w_inverse_identity(back: np.ndarray, M_on_pattern: np.ndarray, relative: bool = False) -> float:
    """Eq. 12: back = f^-1(f(M)) on the pattern of f(M); M_on_pattern is M
    placed in that pattern (zeros where M has no entry)."""
    back = np.asarray(back).ravel()
    M = np.asarray(M_on_pattern).ravel()
    if relative:
        keep = np.abs(M) > 1e-12
        d = (back[keep] - M[keep]) / M[keep]
    else:
        d = back - M
    return float(np.sqrt(np.sum(d * d)) / back.shape[0])
