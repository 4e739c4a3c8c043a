"""Oracle for sampled columns of the truncated chain at any size.

TEST INFRASTRUCTURE (see the package header).

The paper notes that the columns of the Chebyshev matrices obey the
recursion independently (Sec. "Expansion in Chebyshev polynomials"): with
the truncation of Eq. 4 to the pattern P_K by left multiplication,

    T_{k+1}[:, c] = P_K[:, c] o (2 M~ T_k[:, c]) - T_{k-1}[:, c],

and T_k[:, c] lives on the support S_c = {r : (r, c) in P_K} of column c, so
that only the block M~[S_c, S_c] takes part.  One column of the sums of
Eq. 1, sum' c_k T_k[:, c], therefore costs n_pl products with a matrix of
|S_c| rows, whatever the size of M~ — the way to check single outputs of a
chain on 80 000 rows.

Pins: tests/test_oracle_columns.py (a dense pattern, where the columns are
those of T_k(M~) from an eigendecomposition, and the full oracle chain on a
sparse pattern).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .csr import Csr


def chain_column(Mt: Csr, K: Csr, c: int, n_pl: int, coefs: np.ndarray):
    """(support rows S_c, sums [nq, |S_c|]) of column c of sum' coefs[q, k] T_k."""
    coefs = np.atleast_2d(np.asarray(coefs, dtype=np.float64))
    # support of column c = row c of the symmetric pattern
    S = np.asarray(K.ci[K.rp[c]:K.rp[c + 1]], dtype=np.int64)
    M = Mt.to_scipy().tocsr()[S][:, S]
    pos = int(np.searchsorted(S, c))
    t_prev = np.zeros(S.size)
    t_prev[pos] = 1.0                       # T_0 e_c
    acc = 0.5 * coefs[:, :1] * t_prev[None, :]
    if n_pl == 1:
        return S, acc
    t = M @ t_prev                          # T_1 e_c = M~ e_c on S_c
    acc = acc + coefs[:, 1:2] * t[None, :]
    for k in range(1, n_pl - 1):
        t_next = 2.0 * (M @ t) - t_prev
        acc = acc + coefs[:, k + 1:k + 2] * t_next[None, :]
        t_prev, t = t, t_next
    return S, acc
