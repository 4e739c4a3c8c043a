"""Oracle of the learned predictor's input: the 64 statistics of H'.

TEST INFRASTRUCTURE (see the package header).

Written from the definition of the feature vector (features of H' on its
pattern, sizes and physical parameters), one scalar row at a time:
  0 c, 1 w: centre and half width of the Gershgorin interval of H';
  2, 3 bounds of S; 4 kT; 5 kT / w; 6 N_e / n; 7 log n; 8 b / 9;
  9-16 Tr T_k(H~) / n, k = 1..8, H~ = (H' - c) / w, by the truncated chain
      (Eq. 4) on the kernel pattern;
  17-40 counts of d~ = (H'_rr - c) / w in 24 equal bins of [-1, 1]
      (bin = floor((d~ + 1) / 2 * 24), clamped), divided by n;
  41-56 counts of R~ = sum_{s != r} |H'_rs| / w in 16 equal bins of [0, 1]
      (clamped), divided by n;
  57, 58 mean and standard deviation (population) of d~; 59, 60 mean and
      max of R~; 61, 62 min and max of d~;
  63 (mu_0 - c) / w, mu_0 solving N(mu) = N_e for the 9-term expansion of
      the erfc occupation with kT = w / 4 built from the same moments,
      bisection on [c - 5 w, c + 5 w] to |N - N_e| <= 1e-9 max(1, N_e).
Counts are exact integers; the GPU computes the same bins in float64.
"""
from __future__ import annotations

import numpy as np

from . import chebyshev as cb
from .csr import Csr, chebyshev
from .pipeline import scaled


def row_stats(Hp: Csr) -> tuple[np.ndarray, np.ndarray]:
    """Diagonal d_r and off-diagonal absolute row sums R_r of a scalar CSR."""
    n = Hp.n
    d = np.zeros(n)
    R = np.zeros(n)
    for r in range(n):
        for k in range(Hp.rp[r], Hp.rp[r + 1]):
            if Hp.ci[k] == r:
                d[r] = Hp.v[k]
            else:
                R[r] += abs(Hp.v[k])
    return d, R


def features(Hp: Csr, K: Csr, b: int, s_lo: float, s_hi: float, n_e: float, kT: float):
    """(features [64] float64, (g_lo, g_hi)) for H' (scalar CSR) and pattern K."""
    n = Hp.n
    d, R = row_stats(Hp)
    g_lo, g_hi = float(np.min(d - R)), float(np.max(d + R))
    c, w = 0.5 * (g_lo + g_hi), 0.5 * (g_hi - g_lo)
    dt, rt = (d - c) / w, R / w
    bd = np.clip(np.floor((dt + 1.0) * 0.5 * 24).astype(np.int64), 0, 23)
    br = np.clip(np.floor(rt * 16).astype(np.int64), 0, 15)
    hd = np.bincount(bd, minlength=24)
    hr = np.bincount(br, minlength=16)
    _, mom = chebyshev(scaled(Hp, g_lo, g_hi), K, 9, None)
    mu0, _ = cb.bisect_mu(mom, g_lo, g_hi, 0.25 * w, n_e, 1e-9 * max(1.0, n_e),
                          mu_lo=c - 5 * w, mu_hi=c + 5 * w)
    f = np.zeros(64)
    f[0], f[1], f[2], f[3] = c, w, s_lo, s_hi
    f[4], f[5], f[6], f[7], f[8] = kT, kT / w, n_e / n, np.log(n), b / 9.0
    f[9:17] = mom[1:9] / n
    f[17:41] = hd / n
    f[41:57] = hr / n
    f[57], f[58] = dt.mean(), dt.std()
    f[59], f[60] = rt.mean(), rt.max()
    f[61], f[62] = dt.min(), dt.max()
    f[63] = (mu0 - c) / w
    return f, (g_lo, g_hi), (hd, hr)
