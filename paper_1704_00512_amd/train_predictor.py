"""Trains the learned predictor of spectral bounds and mu (CHESS_BOUNDS_LEARNED)
and evaluates it on held-out systems.

    python paper_1704_00512_amd/train_predictor.py collect --train 1000 --data d.npz
    python paper_1704_00512_amd/train_predictor.py fit --data d.npz --test 150

(Run by path: the generator worker processes then load only NumPy/SciPy.)

Data: seeded synthetic systems from workloads.generator.predictor_system,
generated on host worker processes.  For each system, on the GPU through the
library:
  features  chess_features (Gershgorin interval of H', histograms, moments);
  labels    chess_fermi_operator in float64 with Lanczos bounds (no margin),
            tol_fit 1e-10 and two passes: the bounds it used (eps_min,
            eps_max) and the mu it found.
Targets are (label - c) / w in units of the Gershgorin interval.
Training: full-batch Adam on the library's own kernels (chess_mlp_forward /
chess_mlp_grad / chess_mlp_adam), 10 % of the training systems held back to
size the margins: margin = max(0.04, |mean| + 3 std) of the validation
residuals (bounds), mu_half = max(0.02, |mean| + 3 std) of |mu error|.
Evaluation (held-out seeds): the Fermi operator with the learned bounds
against the same call with Gershgorin bounds (the method without the
predictor): terms n_pl, bisection steps, fallbacks, mu and K differences.

Writes the model blob (CHESS_MODEL_FLOATS float32, .npy) and a JSON report.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "predictor_model.npy")
REPORT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "predictor_report.json")


def _log(msg):
    print(f"[train] {msg}", flush=True)


def label_system(ctx, s, want_labels=True):
    import torch
    from paper_1704_00512_amd import BlockPattern, chess_features, chess_fermi_operator
    dev = torch.device("cuda:0")
    H = torch.tensor(s.H, device=dev)
    S = torch.tensor(s.S, device=dev)
    ph = BlockPattern.from_host(s.b, s.pat_h.row_ptr, s.pat_h.col_idx, dev)
    pk = BlockPattern.from_host(s.b, s.pat_k.row_ptr, s.pat_k.col_idx, dev)
    f, g = chess_features(ctx, H, ph, S, ph, pk, s.n_electrons, s.kT, precision="f64")
    lab = None
    if want_labels:
        _, info = chess_fermi_operator(ctx, H, ph, S, ph, pk, s.n_electrons, s.kT, precision="f64",
                                       bounds_mode="lanczos", bound_margin=0.0, tol_fit=1e-10,
                                       store_history=0)
        lab = np.array([info["lo"], info["hi"], info["mu"]])
    return f, np.array(g), lab, (H, S, ph, pk)


def make_pool(workers):
    """Generator workers with single-threaded BLAS (many processes share the
    host cores)."""
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    return mp.get_context("spawn").Pool(workers)


def collect(seeds, pool, with_labels=True, budget_s=None):
    from paper_1704_00512_amd import Context
    from workloads.generator import predictor_system
    feats, gers, labs, systems = [], [], [], []
    t0 = time.time()
    for k, (seed, s) in enumerate(zip(seeds, pool.imap(predictor_system, seeds, chunksize=4))):
        if budget_s is not None and time.time() - t0 > budget_s:
            _log(f"time budget reached after {k} systems")
            break
        ctx = Context(0)
        t1 = time.time()
        try:
            f, g, lab, _ = label_system(ctx, s, with_labels)
        finally:
            ctx.close()
        if k < 5:
            _log(f"system {seed}: n={s.n} b={s.b} kT={s.kT:.4f} {time.time() - t1:.2f} s")
        feats.append(f)
        gers.append(g)
        labs.append(lab)
        systems.append(seed)
        if (k + 1) % 10 == 0:
            _log(f"{k + 1}/{len(seeds)} systems in {time.time() - t0:.0f} s")
    return np.array(feats), np.array(gers), (np.array(labs) if with_labels else None), systems


def targets(gers, labs):
    c = 0.5 * (gers[:, 0] + gers[:, 1])
    w = 0.5 * (gers[:, 1] - gers[:, 0])
    return (labs - c[:, None]) / w[:, None]


def train(X, T, epochs, lr, seed=0):
    """Full-batch Adam on the library kernels; X, T already normalised."""
    import torch
    from paper_1704_00512_amd import Context, chess_mlp_adam, chess_mlp_forward, chess_mlp_grad
    from paper_1704_00512_amd import _lib
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    ni, nh, no = _lib.N_FEATURES, _lib.MLP_HIDDEN, _lib.MLP_OUT
    a1, a2 = np.sqrt(6.0 / (ni + nh)), np.sqrt(6.0 / (nh + no))
    p0 = np.concatenate([rng.uniform(-a1, a1, nh * ni), np.zeros(nh),
                         rng.uniform(-a2, a2, no * nh), np.zeros(no)]).astype(np.float32)
    ctx = Context(0)
    P = torch.tensor(p0, device=dev)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    Xd = torch.tensor(X, dtype=torch.float32, device=dev).contiguous()
    Td = torch.tensor(T, dtype=torch.float32, device=dev).contiguous()
    work = torch.empty(X.shape[0] * (no + nh), dtype=torch.float32, device=dev)
    grad = torch.empty(_lib.MLP_PARAMS, dtype=torch.float32, device=dev)
    losses = []
    for ep in range(1, epochs + 1):
        y, hid = chess_mlp_forward(ctx, P, Xd, want_hidden=True)
        want = ep % 500 == 0 or ep == 1
        _, loss = chess_mlp_grad(ctx, P, Xd, hid, y, Td, work=work, grad=grad, want_loss=want)
        lr_t = lr * 0.5 * (1.0 + np.cos(np.pi * (ep - 1) / epochs)) + 1e-5
        chess_mlp_adam(ctx, P, grad, M, V, ep, lr_t)
        if want:
            losses.append((ep, loss))
            _log(f"epoch {ep}: loss {loss:.3e}")
    p = P.cpu().numpy()
    ctx.close()
    return p, losses


def predict_norm(p, X):
    import torch
    from paper_1704_00512_amd import Context, chess_mlp_forward
    ctx = Context(0)
    y = chess_mlp_forward(ctx, torch.tensor(p, device="cuda"),
                          torch.tensor(X, dtype=torch.float32, device="cuda").contiguous())
    out = y.cpu().numpy().astype(np.float64)
    ctx.close()
    return out


def evaluate(blob, seeds, pool):
    """Learned bounds against Gershgorin bounds on held-out systems."""
    from paper_1704_00512_amd import Context, chess_fermi_operator, chess_model_load
    from workloads.generator import predictor_system
    rows = []
    t0 = time.time()
    for k, (seed, s) in enumerate(zip(seeds, pool.imap(predictor_system, seeds, chunksize=4))):
        ctx = Context(0)
        try:
            chess_model_load(ctx, blob)
            _, _, _, (H, S, ph, pk) = label_system(ctx, s, want_labels=False)
            common = dict(precision="f64", tol_fit=1e-10, store_history=0)
            K_g, ig = chess_fermi_operator(ctx, H, ph, S, ph, pk, s.n_electrons, s.kT,
                                           bounds_mode="gershgorin", **common)
            Kg = K_g.cpu().numpy()
            K_l, il = chess_fermi_operator(ctx, H, ph, S, ph, pk, s.n_electrons, s.kT,
                                           bounds_mode="learned", **common)
            Kl = K_l.cpu().numpy()
        finally:
            ctx.close()
        rows.append(dict(seed=seed, n=s.n, b=s.b, kT=s.kT, n_pl_gersh=ig["n_pl"],
                         n_pl_learned=il["n_pl"], bisect_gersh=ig["bisect_iters"],
                         bisect_learned=il["bisect_iters"], fallback=il["fallback"],
                         mu_gersh=ig["mu"], mu_learned=il["mu"], pred_mu=il["pred_mu"],
                         pred_lo=il["pred_lo"], pred_hi=il["pred_hi"], lo_used=il["lo"],
                         hi_used=il["hi"], gersh_lo=ig["lo"], gersh_hi=ig["hi"],
                         max_abs_dK=float(np.max(np.abs(Kl - Kg))),
                         ms_gersh=ig["ms_total"], ms_learned=il["ms_total"]))
        if (k + 1) % 10 == 0:
            _log(f"evaluated {k + 1}/{len(seeds)} in {time.time() - t0:.0f} s")
    return rows


def summarise(rows):
    a = lambda key: np.array([r[key] for r in rows], dtype=np.float64)
    npg, npl = a("n_pl_gersh"), a("n_pl_learned")
    fb = np.array([r["fallback"] for r in rows])
    return dict(
        systems=len(rows),
        n_pl_ratio_mean=float(np.mean(npg / npl)), n_pl_ratio_median=float(np.median(npg / npl)),
        terms_saved_fraction=float(1.0 - npl.sum() / npg.sum()),
        bisect_iters_gersh_mean=float(a("bisect_gersh").mean()),
        bisect_iters_learned_mean=float(a("bisect_learned").mean()),
        bounds_fallback_rate=float(np.mean((fb & 1) != 0)),
        mu_bracket_miss_rate=float(np.mean((fb & 2) != 0)),
        pred_mu_abs_err_mean=float(np.mean(np.abs(a("pred_mu") - a("mu_gersh")))),
        pred_mu_abs_err_max=float(np.max(np.abs(a("pred_mu") - a("mu_gersh")))),
        mu_diff_max=float(np.max(np.abs(a("mu_learned") - a("mu_gersh")))),
        max_abs_dK=float(np.max(a("max_abs_dK"))),
        time_ratio_mean=float(np.mean(a("ms_gersh") / a("ms_learned"))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("stage", choices=["collect", "fit"])
    ap.add_argument("--train", type=int, default=1000)
    ap.add_argument("--test", type=int, default=150)
    ap.add_argument("--epochs", type=int, default=6000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--data", required=True, help="features and labels (.npz)")
    ap.add_argument("--budget", type=float, default=None,
                    help="collect: stop after this many seconds (keeps what was collected)")
    ap.add_argument("--out", default=MODEL_PATH)
    ap.add_argument("--report", default=REPORT_PATH)
    args = ap.parse_args()
    from paper_1704_00512_amd import _lib
    from workloads.generator import PREDICTOR_TEST_SEED0, PREDICTOR_TRAIN_SEED0

    if args.stage == "collect":
        with make_pool(args.workers) as pool:
            _log(f"features and labels of {args.train} training systems")
            tr_seeds = [PREDICTOR_TRAIN_SEED0 + i for i in range(args.train)]
            X, G, L, seeds = collect(tr_seeds, pool, budget_s=args.budget)
        np.savez(args.data, X=X, G=G, L=L, seeds=np.array(seeds))
        _log(f"data written to {args.data}")
        return
    d = np.load(args.data)
    X, G, L = d["X"], d["G"], d["L"]
    T = targets(G, L)
    ntr = X.shape[0]
    nval = max(1, ntr // 10)
    Xtr, Ttr, Xva, Tva = X[nval:], T[nval:], X[:nval], T[:nval]
    x_mean = Xtr.mean(axis=0)
    x_std = np.maximum(Xtr.std(axis=0), 1e-6)
    y_mean = Ttr.mean(axis=0)
    y_std = np.maximum(Ttr.std(axis=0), 1e-6)
    p, losses = train((Xtr - x_mean) / x_std, (Ttr - y_mean) / y_std, args.epochs, args.lr)
    Yva = predict_norm(p, (Xva - x_mean) / x_std) * y_std + y_mean
    r = Yva - Tva  # residuals in Gershgorin half widths
    margin_lo = max(0.04, abs(r[:, 0].mean()) + 3 * r[:, 0].std())
    margin_hi = max(0.04, abs(r[:, 1].mean()) + 3 * r[:, 1].std())
    mu_half = max(0.02, abs(r[:, 2].mean()) + 3 * r[:, 2].std())
    _log(f"validation residual std: lo {r[:, 0].std():.4f} hi {r[:, 1].std():.4f} "
         f"mu {r[:, 2].std():.4f}; margins {margin_lo:.4f} {margin_hi:.4f} mu_half {mu_half:.4f}")
    norm = np.concatenate([x_mean, 1.0 / x_std, y_mean, y_std])
    blob = np.concatenate([norm, [margin_lo, margin_hi, mu_half], p]).astype(np.float32)
    assert blob.size == _lib.MODEL_FLOATS
    np.save(args.out, blob)
    _log(f"model written to {args.out}")
    with make_pool(args.workers) as pool:
        te_seeds = [PREDICTOR_TEST_SEED0 + i for i in range(args.test)]
        rows = evaluate(blob, te_seeds, pool)
    rep = dict(train_systems=ntr - nval, validation_systems=nval, epochs=args.epochs,
               lr=args.lr, final_loss=losses[-1][1], losses=losses,
               validation_residual_std=[float(v) for v in r.std(axis=0)],
               margins=[margin_lo, margin_hi, mu_half], held_out=summarise(rows), rows=rows)
    with open(args.report, "w") as fh:
        json.dump(rep, fh, indent=1)
    _log("held-out: " + json.dumps(rep["held_out"]))


if __name__ == "__main__":
    main()
