"""Pins of the column oracle (oracle/columns.py): on a dense pattern the
columns are those of sum' c_k T_k(M~) from an eigendecomposition (no
truncation); on a sparse pattern they equal the columns of the oracle's own
full-matrix chain (csr_chain.c, a different code path)."""
import numpy as np

from oracle import columns as oc
from oracle import pipeline as opl
from oracle.csr import Csr, chebyshev
from workloads import generator as g


def test_dense_pattern_columns_match_eigendecomposition():
    rng = np.random.default_rng(0)
    n = 30
    A = rng.standard_normal((n, n))
    A = 0.5 * (A + A.T)
    w, V = np.linalg.eigh(A)
    A = A / (1.05 * np.max(np.abs(w)))     # spectrum inside [-1, 1]
    w, V = np.linalg.eigh(A)
    dense = Csr(n, np.arange(0, n * n + 1, n), np.tile(np.arange(n), n), A.ravel())
    n_pl = 25
    coefs = rng.standard_normal((2, n_pl)) / np.arange(1, n_pl + 1)
    theta = np.arccos(np.clip(w, -1, 1))
    for q in range(2):
        fw = 0.5 * coefs[q, 0] + sum(coefs[q, k] * np.cos(k * theta) for k in range(1, n_pl))
        P = (V * fw) @ V.T
        for c in (0, 7, n - 1):
            S, acc = oc.chain_column(dense, dense, c, n_pl, coefs)
            assert np.array_equal(S, np.arange(n))
            assert np.max(np.abs(acc[q] - P[:, c])) < 1e-12


def test_sparse_pattern_columns_match_full_oracle_chain():
    s = g.make_system(40, 4, 4.6, 6.2, seed=3)
    H = opl.BlockMat(s.pat_h.nb, s.b, s.pat_h.row_ptr, s.pat_h.col_idx, s.H)
    P = opl.BlockMat(s.pat_k.nb, s.b, s.pat_k.row_ptr, s.pat_k.col_idx)
    Mt = opl.scaled(H.csr(), -3.0, 0.2)
    K = P.pattern_csr()
    n_pl = 33
    coefs = np.random.default_rng(1).standard_normal((2, n_pl)) / np.arange(1, n_pl + 1)
    acc, _ = chebyshev(Mt, K, n_pl, coefs)
    full = [K.with_values(acc[q]).dense() for q in range(2)]
    for c in (0, 13, 77, K.n - 1):
        S, col = oc.chain_column(Mt, K, c, n_pl, coefs)
        for q in range(2):
            ref = full[q][:, c]
            assert np.max(np.abs(col[q] - ref[S])) < 1e-13
            # nothing outside the column's support
            mask = np.ones(K.n, bool)
            mask[S] = False
            assert np.all(ref[mask] == 0.0)
