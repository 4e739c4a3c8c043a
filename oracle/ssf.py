"""Oracle for the Segment Storage Format (Sec. "Storage format of the sparse
matrices"): conversion between SSF and block CSR through a dense matrix.

TEST INFRASTRUCTURE (see the package header).

SSF stores the non-zero entries of a sparse n x n matrix as nseg segments of
consecutive entries, one 1-D value array, and two descriptors: keyg(2,2,nseg)
with (c_s, c_e; r_s, r_e), the start and end column and row of each segment
in dense coordinates, and keyv(nseg), where each segment starts in the value
array (redundant: it follows from keyg).  Readings: indices are 1-based (the
format comes from Fortran); the storage is by rows, a segment running in
row-major order from (r_s, c_s) to (r_e, c_e); keyg is given here as an
[nseg, 4] array (c_s, c_e, r_s, r_e).  Exported segments stay within one row
and are maximal runs of consecutive non-zero block columns.

Pins: tests/test_oracle_ssf.py (hand-worked 5 x 5 example, round trips,
brute force, the descriptor count 4 nseg against n + nnz of CRS).
"""
from __future__ import annotations

import numpy as np


def ssf_to_dense(n: int, keyg: np.ndarray, keyv: np.ndarray | None, val: np.ndarray):
    """Dense values and a dense mask of stored entries."""
    keyg = np.asarray(keyg, dtype=np.int64).reshape(-1, 4)
    D = np.zeros((n, n))
    M = np.zeros((n, n), dtype=bool)
    pos = 0
    for s, (cs, ce, rs, re_) in enumerate(keyg):
        a = (rs - 1) * n + (cs - 1)          # row-major dense index of the first entry
        e = (re_ - 1) * n + (ce - 1)
        length = e - a + 1
        start = pos if keyv is None else int(keyv[s]) - 1
        for k in range(length):
            r, c = divmod(a + k, n)
            D[r, c] = val[start + k]
            M[r, c] = True
        pos = start + length
    return D, M


def dense_to_bcsr(D: np.ndarray, M: np.ndarray, b: int):
    """Block pattern: block (I, J) stored when any entry of it is stored."""
    nb = D.shape[0] // b
    rp = [0]
    ci, vals = [], []
    for I in range(nb):
        for J in range(nb):
            if M[I * b:(I + 1) * b, J * b:(J + 1) * b].any():
                ci.append(J)
                vals.append(D[I * b:(I + 1) * b, J * b:(J + 1) * b].copy())
        rp.append(len(ci))
    return (np.array(rp, dtype=np.int64), np.array(ci, dtype=np.int32),
            np.array(vals).reshape(-1, b, b) if vals else np.zeros((0, b, b)))


def bcsr_to_dense(nb: int, b: int, rp, ci, val):
    n = nb * b
    D = np.zeros((n, n))
    M = np.zeros((n, n), dtype=bool)
    for I in range(nb):
        for q in range(rp[I], rp[I + 1]):
            J = ci[q]
            D[I * b:(I + 1) * b, J * b:(J + 1) * b] = val[q]
            M[I * b:(I + 1) * b, J * b:(J + 1) * b] = True
    return D, M


def dense_to_ssf(D: np.ndarray, M: np.ndarray):
    """Segments per row: maximal runs of stored entries."""
    n = D.shape[0]
    keyg, keyv, val = [], [], []
    for r in range(n):
        c = 0
        while c < n:
            if not M[r, c]:
                c += 1
                continue
            c0 = c
            while c < n and M[r, c]:
                c += 1
            keyg.append((c0 + 1, c, r + 1, r + 1))
            keyv.append(len(val) + 1)
            val.extend(D[r, c0:c])
    return (np.array(keyg, dtype=np.int64).reshape(-1, 4), np.array(keyv, dtype=np.int64),
            np.array(val, dtype=np.float64))
