"""Trains the learned predictor of spectral bounds and mu (CHESS_BOUNDS_LEARNED
and CHESS_BOUNDS_LEARNED_LANCZOS) and evaluates it on held-out systems.

    python paper_1704_00512_amd/train_predictor.py collect --start 0 --count 500 --data d0.npz
    python paper_1704_00512_amd/train_predictor.py fit --data d0.npz d1.npz ...
    python paper_1704_00512_amd/train_predictor.py evaluate --start 0 --count 100 --rows e0.json
    python paper_1704_00512_amd/train_predictor.py report --rows e0.json e1.json ...

(Run by path: the generator worker processes then load only NumPy/SciPy.
collect and evaluate take seed ranges so that a large set can be built in
several runs.)

Data: seeded synthetic systems from workloads.generator.predictor_system
(500-3000 atoms, b = 4 or 9, onsite mean -0.5 +- 0.3 Ha, hopping scale
0.2-0.4, kT 0.002-0.02 Ha), generated on host worker processes.  For each
system, on the GPU through the library:
  features  chess_features (Gershgorin interval of H', histograms, moments);
  labels    chess_fermi_operator with Lanczos bounds (no margin): the bounds
            it used after the Eq. 6 / growth checks (eps_min, eps_max) and
            the mu it found; float32 chains with tol_fit 1e-7 by default
            (float64 chains with tol_fit 1e-10 cost 5-10x more on the 9x9
            systems), with the first --check-f64 systems of each run also
            labelled in float64 to measure the difference.
Targets are (label - c) / w in units of the Gershgorin interval.
Training: full-batch Adam on the library's own kernels (chess_mlp_forward /
chess_mlp_grad / chess_mlp_adam), 10 % of the training systems held back to
size the margins from one-sided residual quantiles: margin_lo is the 0.99
quantile of (predicted - label) for eps_min, margin_hi that of (label -
predicted) for eps_max, mu_half that of |predicted mu - mu|.
Evaluation (held-out seeds, float32 chains, tol_fit 1e-6 as in the large
benchmark): the Fermi operator with each bounds mode - Gershgorin (the
method without any estimate), Lanczos, the predictor alone, and the
predictor intersected with Lanczos - reporting terms n_pl, bisection steps,
fallbacks, time, and the K and mu differences against the Lanczos form (the
Gershgorin form, several times the terms, runs on every fifth system).

Writes the model blob (CHESS_MODEL_FLOATS float32, .npy) and a JSON report.
"""
from __future__ import annotations

import argparse
import functools
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
N_MIN, N_MAX = 500, 3000
MODES = ("gershgorin", "lanczos", "learned", "learned_lanczos")


def _log(msg):
    print(f"[train] {msg}", flush=True)


def device_system(s):
    import torch
    from paper_1704_00512_amd import BlockPattern
    dev = torch.device("cuda:0")
    H = torch.tensor(s.H, device=dev)
    S = torch.tensor(s.S, device=dev)
    ph = BlockPattern.from_host(s.b, s.pat_h.row_ptr, s.pat_h.col_idx, dev)
    pk = BlockPattern.from_host(s.b, s.pat_k.row_ptr, s.pat_k.col_idx, dev)
    return H, S, ph, pk


LABEL_FORMS = {"f32": dict(precision="f32", tol_fit=1e-7),
               "f64": dict(precision="f64", tol_fit=1e-10)}


def label_system(ctx, s, precisions=("f32",)):
    """Features, Gershgorin interval and one label (lo, hi, mu) per precision."""
    from paper_1704_00512_amd import chess_features, chess_fermi_operator
    H, S, ph, pk = device_system(s)
    f, g = chess_features(ctx, H, ph, S, ph, pk, s.n_electrons, s.kT, precision="f64")
    labs = []
    for p in precisions:
        _, info = chess_fermi_operator(ctx, H, ph, S, ph, pk, s.n_electrons, s.kT,
                                       bounds_mode="lanczos", bound_margin=0.0, store_history=1,
                                       **LABEL_FORMS[p])
        labs.append(np.array([info["lo"], info["hi"], info["mu"]]))
    return f, np.array(g), labs


def make_pool(workers):
    """Generator workers with single-threaded BLAS (many processes share the
    host cores)."""
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    return mp.get_context("spawn").Pool(workers)


def systems(pool, seeds):
    from workloads.generator import predictor_system
    gen = functools.partial(predictor_system, n_min=N_MIN, n_max=N_MAX)
    return zip(seeds, pool.imap(gen, seeds, chunksize=2))


def collect(seeds, pool, budget_s=None, label="f32", check_f64=0):
    from paper_1704_00512_amd import Context
    feats, gers, labs, done, checks = [], [], [], [], []
    t0 = time.time()
    ctx = Context(0)
    try:
        for k, (seed, s) in enumerate(systems(pool, seeds)):
            if budget_s is not None and time.time() - t0 > budget_s:
                _log(f"time budget reached after {k} systems")
                break
            check = label != "f64" and k < check_f64
            f, g, ls = label_system(ctx, s, (label, "f64") if check else (label,))
            feats.append(f)
            gers.append(g)
            labs.append(ls[0])
            done.append(seed)
            if check:
                checks.append(np.abs(ls[0] - ls[1]))
            if (k + 1) % 10 == 0:
                _log(f"{k + 1}/{len(seeds)} systems in {time.time() - t0:.0f} s (last n={s.n} b={s.b})")
    finally:
        ctx.close()
    return np.array(feats), np.array(gers), np.array(labs), done, np.array(checks).reshape(-1, 3)


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


def evaluate(blob, seeds, pool, gersh_every=5, budget_s=None, warm=False):
    """Every bounds mode on held-out systems (float32, tol_fit 1e-6); the
    Gershgorin form (several times the terms) on every gersh_every-th system.
    Without warm, the first mode timed on a system also pays for building
    its plans and timing kernel variants; with warm an untimed call does
    that first, so the times compare the modes alone."""
    import torch
    from paper_1704_00512_amd import Context, chess_fermi_operator, chess_model_load
    rows = []
    t0 = time.time()
    ctx = Context(0)
    chess_model_load(ctx, blob)
    try:
        for k, (seed, s) in enumerate(systems(pool, seeds)):
            if budget_s is not None and time.time() - t0 > budget_s:
                _log(f"time budget reached after {k} systems")
                break
            H, S, ph, pk = device_system(s)
            row = dict(seed=seed, n=s.n, b=s.b, kT=s.kT, warm=warm)
            if warm:
                chess_fermi_operator(ctx, H, ph, S, ph, pk, s.n_electrons, s.kT, precision="f32",
                                     tol_fit=1e-6, store_history=1, bounds_mode="lanczos")
            K = {}
            for mode in MODES:
                if mode == "gershgorin" and (seed - seeds[0]) % gersh_every != 0:
                    continue
                torch.cuda.synchronize()
                t = time.perf_counter()
                Km, im = chess_fermi_operator(ctx, H, ph, S, ph, pk, s.n_electrons, s.kT,
                                              precision="f32", tol_fit=1e-6, store_history=1,
                                              bounds_mode=mode)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t) * 1e3
                K[mode] = Km.cpu().numpy()
                row[mode] = dict(n_pl=im["n_pl"], bisect=im["bisect_iters"], passes=im["passes"],
                                 fallback=im["fallback"], mu=im["mu"], lo=im["lo"], hi=im["hi"],
                                 ms=ms, ms_learned=im["ms_learned"],
                                 pred=[im["pred_lo"], im["pred_hi"], im["pred_mu"]])
            for mode in K:
                if mode != "lanczos":
                    row[mode]["max_abs_dK"] = float(np.max(np.abs(K[mode] - K["lanczos"])))
                    row[mode]["dmu"] = abs(row[mode]["mu"] - row["lanczos"]["mu"])
            rows.append(row)
            if (k + 1) % 5 == 0:
                _log(f"evaluated {k + 1}/{len(seeds)} in {time.time() - t0:.0f} s (last n={s.n} b={s.b})")
    finally:
        ctx.close()
    return rows


def summarise(rows):
    """Per mode over all systems; ratios to the Gershgorin form over the
    systems where it ran; K and mu differences against the Lanczos form."""
    out = dict(systems=len(rows), form="float32 chain, tol_fit 1e-6, T_k stored (one chain pass "
                                        "when they fit)",
               differences="K and mu against the Lanczos form of the same system")
    sub = [r for r in rows if "gershgorin" in r]
    for mode in MODES:
        have = [r for r in rows if mode in r]
        a = lambda key, rs=have: np.array([r[mode][key] for r in rs], dtype=np.float64)
        d = dict(systems=len(have), n_pl_mean=float(a("n_pl").mean()),
                 n_pl_median=float(np.median(a("n_pl"))), bisect_mean=float(a("bisect").mean()),
                 passes_mean=float(a("passes").mean()), ms_mean=float(a("ms").mean()),
                 ms_median=float(np.median(a("ms"))))
        if sub:
            g = lambda key: np.array([r["gershgorin"][key] for r in sub], dtype=np.float64)
            m = lambda key: np.array([r[mode][key] for r in sub], dtype=np.float64)
            d.update(terms_vs_gershgorin=float(m("n_pl").sum() / g("n_pl").sum()),
                     time_vs_gershgorin=float(m("ms").sum() / g("ms").sum()),
                     time_vs_gershgorin_median=float(np.median(m("ms") / g("ms"))))
        if mode != "lanczos":
            lz = np.array([r["lanczos"]["ms"] for r in have])
            d.update(time_vs_lanczos_median=float(np.median(a("ms") / lz)))
        if mode != "lanczos":
            d.update(max_abs_dK=float(a("max_abs_dK").max()), max_dmu=float(a("dmu").max()))
        if mode.startswith("learned"):
            fb = np.array([r[mode]["fallback"] for r in have])
            pmu = np.array([r[mode]["pred"][2] for r in have])
            mu = np.array([r["lanczos"]["mu"] for r in have])
            d.update(bounds_fallback_rate=float(np.mean((fb & 1) != 0)),
                     mu_bracket_miss_rate=float(np.mean((fb & 2) != 0)),
                     pred_mu_abs_err_mean=float(np.mean(np.abs(pmu - mu))),
                     pred_mu_abs_err_max=float(np.max(np.abs(pmu - mu))),
                     ms_learned_mean=float(a("ms_learned").mean()))
        out[mode] = d
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("stage", choices=["collect", "fit", "evaluate", "report"])
    ap.add_argument("--start", type=int, default=0, help="collect/evaluate: first seed offset")
    ap.add_argument("--count", type=int, default=100, help="collect/evaluate: number of systems")
    ap.add_argument("--epochs", type=int, default=6000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--data", nargs="+", help="features and labels (.npz), one or more")
    ap.add_argument("--rows", nargs="+", help="evaluation rows (.json), one or more")
    ap.add_argument("--label", default="f32", choices=("f32", "f64"), help="collect: label precision")
    ap.add_argument("--check-f64", type=int, default=0,
                    help="collect: also label the first N systems in float64 (label differences)")
    ap.add_argument("--warm", action="store_true",
                    help="evaluate: an untimed call per system first (plans, kernel timing)")
    ap.add_argument("--gersh-every", type=int, default=5,
                    help="evaluate: run the Gershgorin form on every N-th system")
    ap.add_argument("--budget", type=float, default=None,
                    help="collect, evaluate: stop after this many seconds (keeps what was done)")
    ap.add_argument("--out", default=MODEL_PATH)
    ap.add_argument("--report", default=REPORT_PATH)
    args = ap.parse_args()
    from paper_1704_00512_amd import _lib
    from workloads.generator import PREDICTOR_TEST_SEED0, PREDICTOR_TRAIN_SEED0

    if args.stage == "collect":
        seeds = [PREDICTOR_TRAIN_SEED0 + args.start + i for i in range(args.count)]
        with make_pool(args.workers) as pool:
            _log(f"features and labels of training seeds {seeds[0]}..{seeds[-1]}")
            X, G, L, done, chk = collect(seeds, pool, budget_s=args.budget, label=args.label,
                                         check_f64=args.check_f64)
        np.savez(args.data[0], X=X, G=G, L=L, seeds=np.array(done), label=args.label, check_f64=chk)
        if chk.size:
            _log(f"label {args.label} vs float64 on {len(chk)} systems: max |d lo| {chk[:, 0].max():.2e}, "
                 f"|d hi| {chk[:, 1].max():.2e}, |d mu| {chk[:, 2].max():.2e}")
        _log(f"{len(done)} systems written to {args.data[0]}")
        return
    if args.stage == "evaluate":
        seeds = [PREDICTOR_TEST_SEED0 + args.start + i for i in range(args.count)]
        with make_pool(args.workers) as pool:
            rows = evaluate(np.load(args.out), seeds, pool, args.gersh_every, args.budget, args.warm)
        with open(args.rows[0], "w") as fh:
            json.dump(rows, fh)
        _log(f"{len(rows)} rows written to {args.rows[0]}")
        return
    if args.stage == "report":
        rows = []
        for path in args.rows:
            rows += json.load(open(path))
        rows.sort(key=lambda r: (r.get("warm", False), r["seed"]))
        cold = [r for r in rows if not r.get("warm", False)]
        warm = [r for r in rows if r.get("warm", False)]
        rep = json.load(open(args.report)) if os.path.exists(args.report) else {}
        if cold:
            rep["held_out"] = summarise(cold)
            rep["held_out"]["note"] = ("times include, for the first mode run on each system, its "
                                       "plans and kernel-variant timing; see held_out_timing")
        if warm:
            rep["held_out_timing"] = summarise(warm)
            rep["held_out_timing"]["note"] = "after an untimed warm-up call per system"
        rep["rows"] = rows
        with open(args.report, "w") as fh:
            json.dump(rep, fh, indent=1)
        _log("held-out: " + json.dumps(rep["held_out"]))
        return
    parts = [np.load(p) for p in args.data]
    X = np.concatenate([d["X"] for d in parts])
    G = np.concatenate([d["G"] for d in parts])
    L = np.concatenate([d["L"] for d in parts])
    seeds = np.concatenate([d["seeds"] for d in parts])
    order = np.argsort(seeds)
    X, G, L, seeds = X[order], G[order], L[order], seeds[order]
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
    margin_lo = max(0.0, float(np.quantile(r[:, 0], 0.99)))
    margin_hi = max(0.0, float(np.quantile(-r[:, 1], 0.99)))
    mu_half = float(np.quantile(np.abs(r[:, 2]), 0.99))
    _log(f"validation residual std: lo {r[:, 0].std():.4f} hi {r[:, 1].std():.4f} "
         f"mu {r[:, 2].std():.4f}; margins {margin_lo:.4f} {margin_hi:.4f} mu_half {mu_half:.4f}")
    norm = np.concatenate([x_mean, 1.0 / x_std, y_mean, y_std])
    blob = np.concatenate([norm, [margin_lo, margin_hi, mu_half], p]).astype(np.float32)
    assert blob.size == _lib.MODEL_FLOATS
    np.save(args.out, blob)
    _log(f"model written to {args.out}")
    chk = np.concatenate([d["check_f64"].reshape(-1, 3) for d in parts if "check_f64" in d])
    labels = sorted({str(d["label"]) for d in parts if "label" in d}) or ["f64"]
    rep = dict(train_systems=ntr - nval, validation_systems=nval, atoms=[N_MIN, N_MAX],
               labels=f"{'/'.join(labels)} chains ({', '.join(str(LABEL_FORMS[x]) for x in labels)}), "
                      "Lanczos bounds without margin",
               label_vs_f64=dict(systems=int(len(chk)),
                                 max_abs=[float(v) for v in chk.max(axis=0)] if len(chk) else None),
               epochs=args.epochs, lr=args.lr, final_loss=losses[-1][1], losses=losses,
               validation_residual_std=[float(v) for v in r.std(axis=0)],
               margins=[margin_lo, margin_hi, mu_half],
               margin_rule="one-sided 0.99 quantiles of the validation residuals")
    with open(args.report, "w") as fh:
        json.dump(rep, fh, indent=1)
    _log(f"training report written to {args.report}")


if __name__ == "__main__":
    main()
