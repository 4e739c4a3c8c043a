"""Pins of the SSF oracle (oracle/ssf.py): a 5 x 5 example worked by hand,
segments that run over row ends, round trips, and the descriptor count of
the paper (4 nseg for SSF without keyv against n + nnz for CRS).  CPU only."""
import numpy as np

from oracle import ssf


def test_hand_worked_five_by_five():
    # rows (1-based): 1: cols 1-2; 2: cols 1-3; 3: cols 2-3, 5; 4: col 4; 5: cols 3, 5
    keyg = np.array([(1, 2, 1, 1), (1, 3, 2, 2), (2, 3, 3, 3), (5, 5, 3, 3), (4, 4, 4, 4),
                     (3, 3, 5, 5), (5, 5, 5, 5)])
    val = np.arange(1.0, 12.0)
    D, M = ssf.ssf_to_dense(5, keyg, None, val)
    expect = np.array([[1, 2, 0, 0, 0],
                       [3, 4, 5, 0, 0],
                       [0, 6, 7, 0, 8],
                       [0, 0, 0, 9, 0],
                       [0, 0, 10, 0, 11]], dtype=float)
    assert np.array_equal(D, expect)
    assert np.array_equal(M, expect != 0)
    kg, kv, v = ssf.dense_to_ssf(D, M)
    assert np.array_equal(kg, keyg) and np.array_equal(v, val)
    assert np.array_equal(kv, [1, 3, 6, 8, 9, 10, 11])  # keyv follows from keyg


def test_segment_over_row_end_and_explicit_keyv():
    # one segment from (1, 4) to (2, 2) in row-major order, values given out of order via keyv
    keyg = np.array([(4, 2, 1, 2), (1, 1, 3, 3)])
    keyv = np.array([2, 1])
    val = np.array([9.0, 1.0, 2.0, 3.0, 4.0])
    D, M = ssf.ssf_to_dense(4, keyg, keyv, val)
    assert D[0, 3] == 1.0 and D[1, 0] == 2.0 and D[1, 1] == 3.0 and D[2, 0] == 9.0
    assert M.sum() == 4


def test_round_trip_block_patterns_and_descriptor_count():
    rng = np.random.default_rng(0)
    for b in (1, 4, 9):
        nb = 7
        mask = rng.random((nb, nb)) < 0.35
        mask |= np.eye(nb, dtype=bool)
        rp = np.concatenate([[0], np.cumsum(mask.sum(1))])
        ci = np.nonzero(mask)[1].astype(np.int32)
        val = rng.standard_normal((ci.size, b, b))
        D, M = ssf.bcsr_to_dense(nb, b, rp, ci, val)
        kg, kv, v = ssf.dense_to_ssf(D, M)
        D2, M2 = ssf.ssf_to_dense(nb * b, kg, kv, v)
        assert np.array_equal(D2, D) and np.array_equal(M2, M)
        rp2, ci2, val2 = ssf.dense_to_bcsr(D2, M2, b)
        assert np.array_equal(rp2, rp) and np.array_equal(ci2, ci) and np.array_equal(val2, val)
        # every scalar row of a block row has the same runs: nseg = b * (block runs)
        runs = sum(int(np.sum(np.diff(np.concatenate([[0], mask[I].astype(int), [0]])) == 1)) for I in range(nb))
        assert kg.shape[0] == b * runs
        # the paper's count: SSF needs 4 nseg descriptors, CRS n + nnz; SSF is the
        # smaller one exactly when the average segment is longer than 4 (n aside)
        nnz = int(M.sum())
        assert (4 * kg.shape[0] < nnz) == (nnz / kg.shape[0] > 4)
