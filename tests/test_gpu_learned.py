"""The learned bound / mu predictor on the GPU, through the C interface:
perceptron kernels and features against the oracle, the model entry points,
and what the trained model gains over the method without it (Gershgorin
bounds) on held-out systems."""
import os

import numpy as np
import pytest
import torch

from oracle import features as ofeat
from oracle import mlp as omlp
from oracle import pipeline as opl
from paper_1704_00512_amd import (BlockPattern, ChessError, Context, _lib, chess_features,
                                  chess_fermi_operator, chess_mlp_adam, chess_mlp_forward,
                                  chess_mlp_grad, chess_model_load, chess_model_save)
from workloads import generator as g

pytestmark = pytest.mark.gpu

MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_1704_00512_amd", "predictor_model.npy")


def dev(x, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def rand_net(seed, B):
    rng = np.random.default_rng(seed)
    p = (rng.standard_normal(omlp.n_params()) * 0.15).astype(np.float32)
    X = rng.standard_normal((B, 64)).astype(np.float32)
    T = rng.standard_normal((B, 3)).astype(np.float32)
    return p, X, T


@pytest.mark.parametrize("B", [1, 37, 300])
def test_mlp_forward_and_gradient_match_oracle(gpu_ctx, B):
    p, X, T = rand_net(B, B)
    y, hid = chess_mlp_forward(gpu_ctx, dev(p), dev(X), want_hidden=True)
    H_o, Y_o = omlp.forward(p.astype(np.float64), X)
    assert np.max(np.abs(hid.cpu().numpy() - H_o)) < 1e-5
    assert np.max(np.abs(y.cpu().numpy() - Y_o)) < 1e-5
    grad, loss = chess_mlp_grad(gpu_ctx, dev(p), dev(X), hid, y, dev(T))
    g_o = omlp.loss_grad(p.astype(np.float64), X, T)
    scale = max(1.0, np.max(np.abs(g_o)))
    assert np.max(np.abs(grad.cpu().numpy() - g_o)) < 1e-5 * scale
    assert abs(loss - omlp.loss(p.astype(np.float64), X, T)) < 1e-5 * max(1.0, loss)


def test_mlp_normalisation_block(gpu_ctx):
    p, X, _ = rand_net(3, 9)
    rng = np.random.default_rng(4)
    xm, xs = rng.standard_normal(64), rng.uniform(0.5, 2.0, 64)
    ym, ys = rng.standard_normal(3), rng.uniform(0.5, 2.0, 3)
    norm = np.concatenate([xm, 1.0 / xs, ym, ys]).astype(np.float32)
    y = chess_mlp_forward(gpu_ctx, dev(p), dev(X), norm=dev(norm)).cpu().numpy()
    xn = (X.astype(np.float64) - norm[:64]) * norm[64:128]
    _, Yn = omlp.forward(p.astype(np.float64), xn)
    assert np.max(np.abs(y - (Yn * norm[131:134] + norm[128:131]))) < 1e-5 * max(1, np.abs(y).max())


def test_adam_steps_match_oracle(gpu_ctx):
    p, X, T = rand_net(5, 20)
    P, M, V = dev(p), torch.zeros(p.size, device="cuda"), torch.zeros(p.size, device="cuda")
    po, mo, vo = p.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    for t in range(1, 4):
        y, hid = chess_mlp_forward(gpu_ctx, P, dev(X), want_hidden=True)
        grad, _ = chess_mlp_grad(gpu_ctx, P, dev(X), hid, y, dev(T), want_loss=False)
        chess_mlp_adam(gpu_ctx, P, grad, M, V, t, 1e-2)
        # oracle step on the same gradient (the GPU one, so steps stay comparable)
        po, mo, vo = omlp.adam_step(po, grad.cpu().numpy().astype(np.float64), mo, vo, t, 1e-2)
    torch.cuda.synchronize()
    assert np.max(np.abs(P.cpu().numpy() - po)) < 1e-5


def test_features_match_oracle(gpu_ctx):
    s = g.make_system(123, 4, 4.6, 6.2, seed=21, kT=0.01)
    dv = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    ph = BlockPattern.from_host(s.b, s.pat_h.row_ptr, s.pat_h.col_idx)
    pk = BlockPattern.from_host(s.b, s.pat_k.row_ptr, s.pat_k.col_idx)
    sb, nps = (0.25, 2.05), 40
    f, (glo, ghi) = chess_features(gpu_ctx, dv(s.H), ph, dv(s.S), ph, pk, s.n_electrons, s.kT,
                                   precision="f64", s_bounds=sb, n_pl_s=nps)
    bm = lambda p, v=None: opl.BlockMat(p.nb, p.b, p.row_ptr, p.col_idx, v)
    _, Hp, _ = opl.orthogonal_frame(bm(s.pat_h, s.H), bm(s.pat_h, s.S), bm(s.pat_k), sb, nps)
    fo, (olo, ohi), (hd, hr) = ofeat.features(Hp, bm(s.pat_k).pattern_csr(), s.b, sb[0], sb[1],
                                              s.n_electrons, s.kT)
    assert abs(glo - olo) < 1e-10 and abs(ghi - ohi) < 1e-10
    # histogram counts exactly (the features hold count / n in float32)
    n = s.n
    assert np.array_equal(np.rint(f[17:57].astype(np.float64) * n).astype(int),
                          np.concatenate([hd, hr]))
    assert np.allclose(f, fo.astype(np.float32), rtol=2e-6, atol=2e-6)


def test_model_entry_points(gpu_ctx):
    with pytest.raises(ChessError):
        chess_model_load(gpu_ctx, np.zeros(10, dtype=np.float32))
    bad = np.ones(_lib.MODEL_FLOATS, dtype=np.float32)
    bad[5] = np.nan
    with pytest.raises(ChessError):
        chess_model_load(gpu_ctx, bad)
    blob = np.load(MODEL)
    assert blob.dtype == np.float32 and blob.size == _lib.MODEL_FLOATS
    chess_model_load(gpu_ctx, blob)
    assert np.array_equal(chess_model_save(gpu_ctx), blob)


def test_learned_bounds_without_a_model_is_an_error():
    ctx = Context(0)
    s = g.make_system(30, 4, 4.6, 6.2, seed=3, kT=0.02)
    dv = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    ph = BlockPattern.from_host(s.b, s.pat_h.row_ptr, s.pat_h.col_idx)
    pk = BlockPattern.from_host(s.b, s.pat_k.row_ptr, s.pat_k.col_idx)
    with pytest.raises(ChessError):
        chess_fermi_operator(ctx, dv(s.H), ph, dv(s.S), ph, pk, s.n_electrons, s.kT,
                             bounds_mode="learned")
    ctx.close()


def test_learned_predictor_gain_on_held_out_systems():
    """Held-out seeds (never trained on): the learned bounds cut the terms,
    and the result is that of the method without the predictor."""
    blob = np.load(MODEL)
    ratios, bis_l, bis_g, fallbacks = [], [], [], 0
    for i in range(8):
        # held-out seeds of the training distribution, at its small end
        s = g.predictor_system(g.PREDICTOR_TEST_SEED0 + 1000 + i, n_min=500, n_max=1000)
        print(f"[learned] held-out seed {g.PREDICTOR_TEST_SEED0 + 1000 + i} n={s.n} kT={s.kT:.4f}",
              flush=True)
        ctx = Context(0)
        chess_model_load(ctx, blob)
        dv = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
        ph = BlockPattern.from_host(s.b, s.pat_h.row_ptr, s.pat_h.col_idx)
        pk = BlockPattern.from_host(s.b, s.pat_k.row_ptr, s.pat_k.col_idx)
        H, S = dv(s.H), dv(s.S)
        common = dict(precision="f64", tol_fit=1e-10, store_history=1)
        Kg, ig = chess_fermi_operator(ctx, H, ph, S, ph, pk, s.n_electrons, s.kT,
                                      bounds_mode="gershgorin", **common)
        Kl, il = chess_fermi_operator(ctx, H, ph, S, ph, pk, s.n_electrons, s.kT,
                                      bounds_mode="learned", **common)
        ctx.close()
        assert abs(il["mu"] - ig["mu"]) < 1e-7
        assert np.max(np.abs(Kl.cpu().numpy() - Kg.cpu().numpy())) < 1e-6
        assert il["lo"] >= ig["lo"] and il["hi"] <= ig["hi"]
        ratios.append(ig["n_pl"] / il["n_pl"])
        bis_l.append(il["bisect_iters"])
        bis_g.append(ig["bisect_iters"])
        fallbacks += int(il["fallback"] != 0)
    print(f"[learned] n_pl ratio {np.mean(ratios):.2f}, bisection {np.mean(bis_g):.1f} -> "
          f"{np.mean(bis_l):.1f}, fallbacks {fallbacks}/8", flush=True)
    assert np.mean(ratios) > 1.5
    assert np.mean(bis_l) < np.mean(bis_g)
    assert fallbacks <= 2


def test_learned_lanczos_bounds_are_the_intersection(gpu_ctx):
    """CHESS_BOUNDS_LEARNED_LANCZOS: each side from the tighter of the
    predictor's interval and the Lanczos one (when neither is rejected), and
    the result that of the Lanczos form."""
    chess_model_load(gpu_ctx, np.load(MODEL))
    for i in range(3):
        s = g.predictor_system(g.PREDICTOR_TEST_SEED0 + 2000 + i, n_min=500, n_max=700)
        print(f"[learned] intersection, seed {g.PREDICTOR_TEST_SEED0 + 2000 + i} n={s.n}", flush=True)
        dv = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
        ph = BlockPattern.from_host(s.b, s.pat_h.row_ptr, s.pat_h.col_idx)
        pk = BlockPattern.from_host(s.b, s.pat_k.row_ptr, s.pat_k.col_idx)
        H, S = dv(s.H), dv(s.S)
        common = dict(precision="f64", tol_fit=1e-10, store_history=1)
        run = lambda mode: chess_fermi_operator(gpu_ctx, H, ph, S, ph, pk, s.n_electrons, s.kT,
                                                bounds_mode=mode, **common)
        K_lz, i_lz = run("lanczos")
        _, i_le = run("learned")
        K_ll, i_ll = run("learned_lanczos")
        assert i_lz["reexpansions"] == 0
        if i_le["fallback"] & 1 == 0 and i_ll["fallback"] & 1 == 0 and i_ll["reexpansions"] == 0:
            assert i_ll["lo"] == max(i_le["lo"], i_lz["lo"])
            assert i_ll["hi"] == min(i_le["hi"], i_lz["hi"])
        assert i_ll["pred_mu"] == i_le["pred_mu"]
        # two converged expansions on different intervals: after truncation to
        # the pattern their K differ by ~1e-7 (as for learned vs Gershgorin)
        assert abs(i_ll["mu"] - i_lz["mu"]) < 1e-7
        assert np.max(np.abs(K_ll.cpu().numpy() - K_lz.cpu().numpy())) < 1e-6
