"""The allocation-free gradient entry point (chess_mlp_grad_noalloc) against
the allocating one (chess_mlp_grad) through the C interface: the same
kernels on the same inputs, so the results must be bitwise equal - on two
calls in a row, the second with a smaller batch (the fixed workspace keeps
the first call's contents), and with the size limit enforced."""
import numpy as np
import pytest
import torch

from paper_1704_00512_amd import (ChessError, chess_mlp_forward, chess_mlp_grad,
                                  chess_mlp_grad_noalloc)
from paper_1704_00512_amd import _lib

pytestmark = pytest.mark.gpu


def case(batch, seed):
    rng = np.random.default_rng(seed)
    dev = torch.device("cuda")
    params = torch.tensor(rng.standard_normal(_lib.MLP_PARAMS) * 0.1, dtype=torch.float32, device=dev)
    x = torch.tensor(rng.standard_normal((batch, _lib.N_FEATURES)), dtype=torch.float32, device=dev)
    t = torch.tensor(rng.standard_normal((batch, _lib.MLP_OUT)), dtype=torch.float32, device=dev)
    return params, x, t


def test_noalloc_gradient_equals_the_allocating_one(gpu_ctx):
    for batch, seed in ((1000, 1), (37, 2)):
        print(f"[no-alloc] batch {batch}", flush=True)
        params, x, t = case(batch, seed)
        y, hidden = chess_mlp_forward(gpu_ctx, params, x, want_hidden=True)
        g_ref, l_ref = chess_mlp_grad(gpu_ctx, params, x, hidden, y, t)
        g_na, l_na = chess_mlp_grad_noalloc(gpu_ctx, params, x, hidden, y, t)
        torch.cuda.synchronize()
        assert torch.equal(g_ref, g_na), batch
        assert l_ref == l_na, (batch, l_ref, l_na)
        # without the loss the call only enqueues its kernels
        g2, l2 = chess_mlp_grad_noalloc(gpu_ctx, params, x, hidden, y, t, want_loss=False)
        torch.cuda.synchronize()
        assert l2 is None and torch.equal(g_ref, g2)


def test_noalloc_size_limit(gpu_ctx):
    params, x, t = case(_lib.NOALLOC_MAX_BATCH + 1, 3)
    y, hidden = chess_mlp_forward(gpu_ctx, params, x, want_hidden=True)
    with pytest.raises(ChessError) as e:
        chess_mlp_grad_noalloc(gpu_ctx, params, x, hidden, y, t)
    assert e.value.name == "CHESS_E_ARG" and "CHESS_NOALLOC_MAX_BATCH" in str(e.value)
    params, x, t = case(_lib.NOALLOC_MAX_BATCH, 4)
    y, hidden = chess_mlp_forward(gpu_ctx, params, x, want_hidden=True)
    g_ref, l_ref = chess_mlp_grad(gpu_ctx, params, x, hidden, y, t)
    g_na, l_na = chess_mlp_grad_noalloc(gpu_ctx, params, x, hidden, y, t)
    assert torch.equal(g_ref, g_na) and l_ref == l_na
