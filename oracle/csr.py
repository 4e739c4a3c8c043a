"""Oracle: ctypes access to the plain-C masked chain (csr_chain.c) plus the
block-to-scalar CSR conversion it needs.

TEST INFRASTRUCTURE ONLY (see csr_chain.c).  The shared object is built by
`build_oracle()` with gcc; nothing here touches a GPU.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csr_chain.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build_oracle(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build_oracle()
        L = ctypes.CDLL(_LIB)
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        L.oracle_masked_spgemm.argtypes = [ctypes.c_int64, i64p, i32p, f64p, i64p, i32p, f64p,
                                           i64p, i32p, f64p]
        L.oracle_masked_spgemm.restype = ctypes.c_int
        L.oracle_chebyshev.argtypes = [ctypes.c_int64, i64p, i32p, f64p, i64p, i32p,
                                       ctypes.c_int32, ctypes.c_int32, f64p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_int32]
        L.oracle_chebyshev.restype = ctypes.c_int
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None
        _lib = L
    return _lib


class Csr:
    """Scalar CSR with sorted column indices (int64 row_ptr, int32 col_idx)."""

    def __init__(self, n, rp, ci, v=None):
        self.n = int(n)
        self.rp = np.ascontiguousarray(rp, dtype=np.int64)
        self.ci = np.ascontiguousarray(ci, dtype=np.int32)
        self.v = None if v is None else np.ascontiguousarray(v, dtype=np.float64)

    @property
    def nnz(self):
        return int(self.ci.shape[0])

    def with_values(self, v):
        return Csr(self.n, self.rp, self.ci, v)

    def to_scipy(self):
        return scipy.sparse.csr_matrix((self.v, self.ci, self.rp), shape=(self.n, self.n))

    def dense(self):
        return self.to_scipy().toarray()

    @staticmethod
    def from_scipy(A):
        A = scipy.sparse.csr_matrix(A)
        A.sort_indices()
        return Csr(A.shape[0], A.indptr, A.indices, A.data)

    def values_from_dense(self, M):
        r = np.repeat(np.arange(self.n), np.diff(self.rp))
        return np.ascontiguousarray(M[r, self.ci])


def block_pattern_to_csr(nb: int, b: int, row_ptr, col_idx) -> Csr:
    """Scalar pattern of a block pattern: block (I, J) covers rows I*b..I*b+b-1
    and columns J*b..J*b+b-1.  Scalar entries come out row-sorted."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    cnt = np.diff(row_ptr)
    rp = np.zeros(nb * b + 1, dtype=np.int64)
    rp[1:] = np.cumsum(np.repeat(cnt * b, b))
    ci = np.empty(int(rp[-1]), dtype=np.int32)
    for I in range(nb):
        cols = col_idx[row_ptr[I]:row_ptr[I + 1]]
        scal = (cols[:, None] * b + np.arange(b)[None, :]).ravel()
        for r in range(b):
            s = rp[I * b + r]
            ci[s:s + scal.shape[0]] = scal
    return Csr(nb * b, rp, ci)


def block_values_to_csr(nb: int, b: int, row_ptr, val) -> np.ndarray:
    """Values [nnzb, b, b] (each block row-major) in the order of
    block_pattern_to_csr."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64).reshape(-1, b, b)
    out = []
    for I in range(nb):
        blk = val[row_ptr[I]:row_ptr[I + 1]]  # [m, b, b]
        out.append(np.transpose(blk, (1, 0, 2)).reshape(-1))  # row r: blocks' row r in order
    return np.ascontiguousarray(np.concatenate(out)) if out else np.zeros(0)


def csr_values_to_block(nb: int, b: int, row_ptr, v) -> np.ndarray:
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    out = np.empty((int(row_ptr[-1]), b, b))
    pos = 0
    for I in range(nb):
        m = int(row_ptr[I + 1] - row_ptr[I])
        chunk = np.asarray(v[pos:pos + m * b * b]).reshape(b, m, b)
        out[row_ptr[I]:row_ptr[I + 1]] = np.transpose(chunk, (1, 0, 2))
        pos += m * b * b
    return out


def masked_spgemm(A: Csr, B: Csr, C: Csr) -> np.ndarray:
    """Values of P_C o (A B)."""
    out = np.zeros(C.nnz)
    rc = lib().oracle_masked_spgemm(A.n, A.rp, A.ci, A.v, B.rp, B.ci, B.v, C.rp, C.ci, out)
    if rc != 0:
        raise MemoryError("oracle_masked_spgemm")
    return out


def chebyshev(Mt: Csr, K: Csr, n_pl: int, coefs: np.ndarray | None,
              k_stop: int | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Truncated chain on P_K: returns (acc [nq, nnz_K], moments [n_pl])."""
    coefs = np.zeros((0, n_pl)) if coefs is None else np.atleast_2d(np.asarray(coefs, dtype=np.float64))
    nq = coefs.shape[0]
    coefs = np.ascontiguousarray(coefs)
    acc = np.zeros((nq, K.nnz))
    mom = np.zeros(n_pl)
    ks = n_pl if k_stop is None else int(k_stop)
    rc = lib().oracle_chebyshev(Mt.n, Mt.rp, Mt.ci, Mt.v, K.rp, K.ci, int(n_pl), int(nq),
                                coefs if nq else np.zeros(1),
                                acc.ctypes.data if nq else None, mom.ctypes.data, ks)
    if rc == -2:
        raise ValueError("pattern of M~ is not contained in P_K")
    if rc != 0:
        raise MemoryError("oracle_chebyshev")
    return acc, mom


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    lib().oracle_set_num_threads(int(n))
