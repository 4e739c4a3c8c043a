"""Segment Storage Format conversions of the library (chess_ssf_to_bcsr,
chess_bcsr_to_ssf, host code behind the C interface) against the oracle
(oracle/ssf.py): bit-exact patterns, descriptors and values for the paper's
workload patterns and random ones, row-spanning segments, explicit keyv,
empty inputs and every error the interface defines."""
import numpy as np
import pytest

from oracle import ssf as ossf
from paper_1704_00512_amd import ChessError, chess_bcsr_to_ssf, chess_ssf_to_bcsr
from workloads import generator as g

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("spec", [(123, 4, 4.6, 6.2, 21), (61, 9, 4.6, 6.2, 22)])
def test_workload_patterns_exact(spec):
    s = g.make_system(*spec[:4], seed=spec[4])
    for pat, vals in ((s.pat_h, s.H), (s.pat_k, None)):
        if vals is None:
            vals = np.random.default_rng(1).standard_normal((pat.nnzb, s.b, s.b))
        kg, kv, v = chess_bcsr_to_ssf(s.b, pat.row_ptr, pat.col_idx, vals)
        D, M = ossf.bcsr_to_dense(pat.nb, s.b, pat.row_ptr, pat.col_idx, vals)
        okg, okv, ov = ossf.dense_to_ssf(D, M)
        assert np.array_equal(kg, okg) and np.array_equal(kv, okv) and np.array_equal(v, ov)
        rp, ci, vb = chess_ssf_to_bcsr(s.b, pat.nb * s.b, kg, v, keyv=kv)
        assert np.array_equal(rp, pat.row_ptr) and np.array_equal(ci, pat.col_idx)
        assert np.array_equal(vb, vals)


def test_random_segments_exact():
    rng = np.random.default_rng(3)
    for b, nb in ((1, 30), (4, 12), (9, 5)):
        n = nb * b
        M = rng.random((n, n)) < 0.2
        D = np.where(M, rng.standard_normal((n, n)), 0.0)
        kg, kv, v = ossf.dense_to_ssf(D, M)
        rp, ci, vb = chess_ssf_to_bcsr(b, n, kg, v)          # keyv omitted
        orp, oci, ovb = ossf.dense_to_bcsr(D, M, b)
        assert np.array_equal(rp, orp) and np.array_equal(ci, oci) and np.array_equal(vb, ovb)


def test_row_spanning_segment_and_explicit_keyv():
    keyg = np.array([(4, 2, 1, 2), (1, 1, 3, 3)])
    keyv = np.array([2, 1])
    val = np.array([9.0, 1.0, 2.0, 3.0, 4.0])
    rp, ci, vb = chess_ssf_to_bcsr(2, 4, keyg, val, keyv=keyv)
    D, M = ossf.ssf_to_dense(4, keyg, keyv, val)
    orp, oci, ovb = ossf.dense_to_bcsr(D, M, 2)
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci) and np.array_equal(vb, ovb)


def test_empty_and_errors():
    rp, ci, vb = chess_ssf_to_bcsr(4, 8, np.zeros((0, 4)), np.zeros(0))
    assert np.array_equal(rp, np.zeros(3)) and ci.size == 0
    kg, kv, v = chess_bcsr_to_ssf(4, np.zeros(3, dtype=np.int64), np.zeros(0), np.zeros((0, 4, 4)))
    assert kg.shape == (0, 4) and v.size == 0
    ok = np.array([(1, 2, 1, 1), (3, 3, 2, 2)])
    bad = [np.array([(0, 2, 1, 1)]),                      # column 0 (1-based)
           np.array([(1, 9, 1, 1)]),                      # past n
           np.array([(3, 1, 1, 1)]),                      # ends before it starts
           np.array([(3, 3, 2, 2), (1, 2, 1, 1)]),        # unsorted
           np.array([(1, 3, 1, 1), (2, 2, 1, 1)])]        # overlapping
    chess_ssf_to_bcsr(2, 4, ok, np.ones(3))
    for kg_bad in bad:
        with pytest.raises(ChessError):
            chess_ssf_to_bcsr(2, 4, kg_bad, np.ones(8))
    with pytest.raises(ChessError):                        # values past the array
        chess_ssf_to_bcsr(2, 4, ok, np.ones(2))
    with pytest.raises(ChessError):                        # n not a multiple of b
        chess_ssf_to_bcsr(3, 4, ok, np.ones(3))
    with pytest.raises(ChessError):                        # columns not increasing
        chess_bcsr_to_ssf(1, np.array([0, 2]), np.array([0, 0]), np.ones((2, 1, 1)))
