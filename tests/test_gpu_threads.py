"""Two contexts on one device, driven from two host threads at once, give the
same results as one context alone.  The library keeps no global state apart
from the launchers' record of raised LDS limits, which is locked; the float64
chain on these cutoffs needs more than 64 KB of LDS per tile, so the threads
run before anything else in this test raises that limit."""
import threading

import numpy as np
import pytest
import torch

from paper_1704_00512_amd import BlockPattern, Context, chess_chebyshev
from workloads import generator as g

pytestmark = pytest.mark.gpu

# the 80 000-row cutoffs on 150 atoms: kernel rows of up to ~150 blocks
SPEC = (150, 4, 5.6, 7.8, 23)


def run(ctx, s, precision):
    ph = BlockPattern.from_host(s.b, s.pat_h.row_ptr, s.pat_h.col_idx)
    pk = BlockPattern.from_host(s.b, s.pat_k.row_ptr, s.pat_k.col_idx)
    H = torch.tensor(s.H, dtype=torch.float64, device="cuda")
    coef = np.random.default_rng(11).standard_normal((2, 40)) / np.arange(1, 41)
    accs, mom = chess_chebyshev(ctx, H, ph, -3.8, 0.2, pk, 40, coef, precision=precision)
    return [a.cpu().numpy() for a in accs], mom


def test_two_threads_two_contexts_match_one(gpu_ctx):
    print(f"[threads] system {SPEC}", flush=True)
    s = g.make_system(*SPEC[:4], seed=SPEC[4])
    precs = ("f64", "f32")
    out = [None, None]
    errs = []

    def work(i):
        try:
            torch.cuda.set_device(0)
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                ctx = Context(0, stream=st)
                try:
                    for _ in range(3):
                        out[i] = run(ctx, s, precs[i])
                finally:
                    ctx.close()
        except Exception as e:  # reported in the main thread
            errs.append(e)

    th = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=90)
    assert not any(t.is_alive() for t in th), "a worker thread did not finish"
    assert not errs, errs
    for i, p in enumerate(precs):
        accs, mom = run(gpu_ctx, s, p)
        assert np.array_equal(mom, out[i][1]), p
        for q in range(2):
            assert np.array_equal(accs[q], out[i][0][q]), (p, q)
