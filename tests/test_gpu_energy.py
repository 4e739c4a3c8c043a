"""Width check of Sec. "Fermi Operator Expansion" (chess_opts.adapt_kt)
through the C interface against the oracle: E = Tr(K' H') and E' for the
wider occupation from the chain's moments, the number of kT halvings and the
returned K, at fixed bounds and degree so that both sides run the same chain.

Bars: float64, |dE| <= 1e-5 - each side finds mu to |N - N_e| <= 1e-8 N_e on
its own (2.5e-6 electrons here), which moves E by about |mu| times that;
float32, |dE| <= 2e-2 - the moments carry float32 rounding, |dt_k| <= 1e-5 n
(the chain bar), and E weights them by |c_k| (1/sigma + |tau|) <= 3.
Decisions are tested only where the oracle's |E - E'| is at least 1.5x away
from the threshold on either side."""
import numpy as np
import pytest
import scipy.linalg
import torch

from oracle import chebyshev as cb
from oracle import pipeline as opl
from oracle.csr import chebyshev
from paper_1704_00512_amd import BlockPattern, chess_fermi_operator
from workloads import generator as g

pytestmark = pytest.mark.gpu

SPEC = (123, 4, 4.6, 6.2, 21)
FIXED = dict(s_bounds=(0.25, 2.05), bounds=(-1.9, 0.1), n_pl=400, n_pl_s=40)
_sys = {}


def system(kT):
    if kT not in _sys:
        print(f"[energy] system {SPEC} kT={kT}", flush=True)
        _sys[kT] = g.make_system(*SPEC[:4], seed=SPEC[4], kT=kT)
    return _sys[kT]


def bm(p, v=None):
    return opl.BlockMat(p.nb, p.b, p.row_ptr, p.col_idx, v)


def dv(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def gpat(p):
    return BlockPattern.from_host(p.b, p.row_ptr, p.col_idx)


def run_gpu(gpu_ctx, s, kT, precision, **kw):
    return chess_fermi_operator(gpu_ctx, dv(s.H), gpat(s.pat_h), dv(s.S), gpat(s.pat_h),
                                gpat(s.pat_k), s.n_electrons, kT, precision=precision,
                                adapt_kt=1, **FIXED, **kw)


def run_oracle(s, kT, **kw):
    return opl.fermi_operator(bm(s.pat_h, s.H), bm(s.pat_h, s.S), bm(s.pat_k), s.n_electrons, kT,
                              s_bounds_=FIXED["s_bounds"], n_pl_s=FIXED["n_pl_s"],
                              h_bounds=FIXED["bounds"], n_pl=FIXED["n_pl"], adapt_kt=True,
                              tol_fit=1e-10, tol_fit_s=1e-10, **kw)


def oracle_k_at(s, info):
    """The oracle's K at the library's final kT and mu (no search, no check)."""
    Ko, _ = opl.fermi_operator(bm(s.pat_h, s.H), bm(s.pat_h, s.S), bm(s.pat_k), s.n_electrons,
                               info["kt_used"], s_bounds_=FIXED["s_bounds"], n_pl_s=FIXED["n_pl_s"],
                               h_bounds=FIXED["bounds"], n_pl=FIXED["n_pl"], mu=info["mu"])
    return Ko


def oracle_differences(s, kT, steps):
    """|E - E'| of the oracle for kT, kT/2, ... (same chain, fixed degree)."""
    _, Hp, _ = opl.orthogonal_frame(bm(s.pat_h, s.H), bm(s.pat_h, s.S), bm(s.pat_k),
                                    FIXED["s_bounds"], FIXED["n_pl_s"], 1e-10)
    lo, hi = FIXED["bounds"]
    n_pl = FIXED["n_pl"]
    _, mom_e = chebyshev(opl.scaled(Hp, lo, hi), bm(s.pat_k).pattern_csr(), n_pl + 1, None)
    mom = mom_e[:n_pl]
    out = []
    for _ in range(steps):
        e = []
        for w in (kT, 1.25 * kT):
            mu, _ = cb.bisect_mu(mom, lo, hi, w, s.n_electrons, 1e-8 * s.n_electrons, "erfc")
            c = cb.cheb_coeffs(lambda x: cb.occ_erfc(x, mu, w), lo, hi, n_pl)
            e.append(cb.energy_from_moments(c, mom_e, lo, hi))
        out.append(abs(e[0] - e[1]))
        kT *= 0.5
    return out


@pytest.mark.parametrize("precision,tol", [("f64", 1e-5), ("f32", 2e-2)])
def test_energies_match_oracle_without_halving(gpu_ctx, precision, tol):
    s = system(0.02)
    K, info = run_gpu(gpu_ctx, s, 0.02, precision, tol_energy=1e9)
    Ko, oi = run_oracle(s, 0.02, tol_energy=1e9)
    assert info["kt_halvings"] == 0 and oi["kt_halvings"] == 0
    assert info["kt_used"] == pytest.approx(0.02)
    assert abs(info["energy"] - oi["energy"]) < tol
    assert abs(info["energy_wide"] - oi["energy_wide"]) < tol
    # K is the expansion at the returned kT and mu (mu of each side is its
    # own bisection, so K is compared with the oracle's at the library's mu)
    assert np.max(np.abs(K.cpu().numpy() - oracle_k_at(s, info))) < (1e-10 if precision == "f64" else 1e-5)


def test_halvings_match_oracle(gpu_ctx):
    s = system(0.16)
    d = oracle_differences(s, 0.16, 4)
    assert d[0] > d[1] > d[2]
    tol_e = float(np.sqrt(d[1] * d[2]))  # two halvings expected: d0, d1 > tol >= d2
    assert d[1] / tol_e >= 1.5 and tol_e / d[2] >= 1.5
    K, info = run_gpu(gpu_ctx, s, 0.16, "f64", tol_energy=tol_e)
    Ko, oi = run_oracle(s, 0.16, tol_energy=tol_e)
    assert oi["kt_halvings"] == 2
    assert info["kt_halvings"] == 2
    assert info["kt_used"] == pytest.approx(0.04)
    assert abs(info["energy"] - oi["energy"]) < 1e-5
    assert np.max(np.abs(K.cpu().numpy() - oracle_k_at(s, info))) < 1e-10
    # the cap on halvings is honoured
    _, info1 = run_gpu(gpu_ctx, s, 0.16, "f64", tol_energy=tol_e, max_kt_halvings=1)
    assert info1["kt_halvings"] == 1 and info1["kt_used"] == pytest.approx(0.08)


def test_homo_lumo_match_oracle(gpu_ctx):
    # the same moments on both sides at fixed bounds and degree; each side
    # bisects to |N - target| <= 1e-10 N_e, about 1e-10 Ha here
    s = system(0.02)
    _, info = chess_fermi_operator(gpu_ctx, dv(s.H), gpat(s.pat_h), dv(s.S), gpat(s.pat_h),
                                   gpat(s.pat_k), s.n_electrons, 0.02, precision="f64",
                                   tol_ne=1e-10, **FIXED)
    _, oinfo = opl.fermi_operator(bm(s.pat_h, s.H), bm(s.pat_h, s.S), bm(s.pat_k), s.n_electrons,
                                  0.02, s_bounds_=FIXED["s_bounds"], n_pl_s=FIXED["n_pl_s"],
                                  h_bounds=FIXED["bounds"], n_pl=FIXED["n_pl"], tol_ne=1e-10)
    assert abs(info["homo"] - oinfo["homo"]) < 1e-8
    assert abs(info["lumo"] - oinfo["lumo"]) < 1e-8
    # N(homo) = N_e - 1/2 < N(mu) = N_e < N(lumo) = N_e + 1/2 and N is increasing
    assert info["homo"] < info["mu"] < info["lumo"]


def sym_blocks(rng, b, centre, spread):
    G = rng.standard_normal((1, b, b))
    return centre * np.eye(b)[None] + spread * 0.5 * (G + np.transpose(G, (0, 2, 1)))


@pytest.mark.parametrize("b,seed,n_e", [(4, 51, 2.0), (9, 52, 4.5)])
def test_homo_lumo_of_isolated_levels_are_the_eigenvalues(gpu_ctx, b, seed, n_e):
    # one atom: levels at least 27 kT apart, so N(e) crosses N - 1/2 exactly at
    # eigenvalue N up to the polynomial error (tol_fit 1e-12); default bounds
    rng = np.random.default_rng(seed)
    H, S = sym_blocks(rng, b, -0.5, 0.2), sym_blocks(rng, b, 1.0, 0.05)
    e = scipy.linalg.eigh(H[0], S[0], eigvals_only=True)
    kT = 2e-3
    assert np.diff(e).min() > 25 * kT
    p = g.pattern_from_pairs(1, b, np.array([0]), np.array([0]))
    _, info = chess_fermi_operator(gpu_ctx, dv(H), gpat(p), dv(S), gpat(p), gpat(p), n_e, kT,
                                   precision="f64", tol_fit=1e-12, tol_fit_s=1e-12)
    nh = int(np.ceil(n_e))
    assert abs(info["homo"] - e[nh - 1]) < 1e-8
    assert abs(info["lumo"] - e[nh]) < 1e-8
    # past the ends of the spectrum
    _, full = chess_fermi_operator(gpu_ctx, dv(H), gpat(p), dv(S), gpat(p), gpat(p), float(b) - 0.5,
                                   kT, precision="f64", tol_fit=1e-12, tol_fit_s=1e-12)
    assert abs(full["homo"] - e[-1]) < 1e-8 and np.isnan(full["lumo"])
