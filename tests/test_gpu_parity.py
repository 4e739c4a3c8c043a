"""Parity of the HIP path (through the C interface) with the oracle.

Tolerances (max-abs): float64 path 1e-10, float32 chain 1e-5; integer-valued
products bit-exact.  Inputs are the seeded synthetic systems of workloads/,
sized so the oracle finishes in seconds while spanning many row tiles and a
ragged last tile.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import torch

from oracle import csr as ocsr
from oracle import dense as odense
from oracle import pipeline as opl
from paper_1704_00512_amd import (BlockPattern, ChessError, chess_chebyshev,
                                  chess_eigs_in_interval, chess_fermi_operator,
                                  chess_masked_product, chess_matrix_power)
from workloads import generator as g

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-10, 1e-5


def gpat(p):
    return BlockPattern.from_host(p.b, p.row_ptr, p.col_idx)


def dt(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def bm(p, val=None):
    return opl.BlockMat(p.nb, p.b, p.row_ptr, p.col_idx, val)


_cache = {}


def system(n_atoms, b, r_h, r_k, seed, kT=0.01):
    key = (n_atoms, b, r_h, r_k, seed, kT)
    if key not in _cache:
        print(f"[gpu-parity] system atoms={n_atoms} b={b} rH={r_h} rK={r_k} seed={seed}", flush=True)
        _cache[key] = g.make_system(n_atoms, b, r_h, r_k, seed=seed, kT=kT)
    return _cache[key]


# 123 atoms: 31 row tiles of 4 with a ragged last tile of 3
SYS4 = (123, 4, 4.6, 6.2, 21)
SYS9 = (61, 9, 4.6, 6.2, 22)
SYSL = (150, 4, 5.6, 7.8, 23)


@pytest.mark.parametrize("spec", [SYS4, SYS9])
def test_masked_product_integer_exact(gpu_ctx, spec):
    s = system(*spec)
    rng = np.random.default_rng(5)
    for pa, pb, pc in ((s.pat_k, s.pat_h, s.pat_k), (s.pat_k, s.pat_k, s.pat_h),
                       (s.pat_h, s.pat_k, s.pat_k)):
        A = rng.integers(-8, 9, (pa.nnzb, s.b, s.b)).astype(np.float64)
        B = rng.integers(-8, 9, (pb.nnzb, s.b, s.b)).astype(np.float64)
        C = chess_masked_product(gpu_ctx, dt(A), gpat(pa), dt(B), gpat(pb), gpat(pc)).cpu().numpy()
        ref = ocsr.masked_spgemm(bm(pa, A).csr(), bm(pb, B).csr(), bm(pc).pattern_csr())
        assert np.array_equal(C, bm(pc).to_block(ref))


def test_masked_product_random_values(gpu_ctx):
    s = system(*SYS4)
    rng = np.random.default_rng(6)
    A = rng.standard_normal((s.pat_k.nnzb, 4, 4))
    B = rng.standard_normal((s.pat_h.nnzb, 4, 4))
    C = chess_masked_product(gpu_ctx, dt(A), gpat(s.pat_k), dt(B), gpat(s.pat_h),
                             gpat(s.pat_k)).cpu().numpy()
    ref = bm(s.pat_k).to_block(ocsr.masked_spgemm(bm(s.pat_k, A).csr(), bm(s.pat_h, B).csr(),
                                                  bm(s.pat_k).pattern_csr()))
    assert np.max(np.abs(C - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def chain_case(gpu_ctx, spec, n_pl, precision, nq=2):
    s = system(*spec)
    # contain the spectrum of H: [-2.78, -0.08] (SYS4), [-3.54, -0.12] (SYSL)
    lo, hi = (-3.8, 0.2) if spec == SYSL else (-3.0, 0.2)
    rng = np.random.default_rng(7)
    coef = rng.standard_normal((nq, n_pl)) / np.arange(1, n_pl + 1)
    accs, mom = chess_chebyshev(gpu_ctx, dt(s.H), gpat(s.pat_h), lo, hi, gpat(s.pat_k), n_pl,
                                coef, precision=precision)
    Mt = opl.scaled(bm(s.pat_h, s.H).csr(), lo, hi)
    acc_o, mom_o = ocsr.chebyshev(Mt, bm(s.pat_k).pattern_csr(), n_pl, coef)
    return s, accs, mom, acc_o, mom_o


@pytest.mark.parametrize("spec", [SYS4, SYS9])
@pytest.mark.parametrize("precision,tol", [("f64", TOL64), ("f32", TOL32)])
def test_chebyshev_chain_parity(gpu_ctx, spec, precision, tol):
    s, accs, mom, acc_o, mom_o = chain_case(gpu_ctx, spec, 60, precision)
    n = s.n
    assert np.max(np.abs(mom - mom_o)) < tol * n
    for q in range(2):
        got = accs[q].cpu().numpy()
        ref = bm(s.pat_k).to_block(acc_o[q])
        assert np.max(np.abs(got - ref)) < tol, (precision, q)


@pytest.mark.parametrize("variant", list(range(27)))
@pytest.mark.parametrize("precision,tol", [("f64", TOL64), ("f32", TOL32)])
def test_chain_kernel_variants(gpu_ctx, monkeypatch, variant, precision, tol):
    # every variant of the b = 4 chain kernel, forced, against the oracle;
    # 24-26 (float32) and 10-12 (float64) are the output-stationary kernel
    monkeypatch.setenv("CHESS_LISTED_VARIANT", str(variant))
    if precision == "f64" and variant in (4, 5) + tuple(range(13, 27)):  # float32-only variants
        with pytest.raises(ChessError):
            chain_case(gpu_ctx, SYS4, 70, precision)
        return
    # SYS4: short hit lists (the remainder loop); SYSL: the cutoffs of the
    # 80 000-row workload, ~70 hits per output block (several pipelined groups)
    # one float64 sum (the kernels specialised for at most one) and two
    for spec in (SYS4, SYSL):
        for nq in (1, 2):
            s, accs, mom, acc_o, mom_o = chain_case(gpu_ctx, spec, 70, precision, nq=nq)
            assert np.max(np.abs(mom - mom_o)) < tol * s.n
            for q in range(nq):
                ref = bm(s.pat_k).to_block(acc_o[q])
                assert np.max(np.abs(accs[q].cpu().numpy() - ref)) < tol, (variant, precision, q, spec)
    s2 = system(*SYS4, kT=0.02)
    _, info = chess_fermi_operator(gpu_ctx, dt(s2.H), gpat(s2.pat_h), dt(s2.S), gpat(s2.pat_h),
                                   gpat(s2.pat_k), s2.n_electrons, s2.kT, precision=precision,
                                   mu=-0.95, **FIX)
    assert info["kernel_variant"] == variant


# dense neighbourhoods: H rows of up to 118 blocks, up to 118 hits per output
# block, so free slot assignment runs up to ~30 rounds per column (32 at most)
SYSD = (200, 4, 6.4, 7.5, 24)


@pytest.mark.parametrize("variant", [12, 16, 18, 20, 21, 24, 25, 26])
def test_chain_kernel_long_hit_lists(gpu_ctx, monkeypatch, variant):
    s = system(*SYSD)
    nb = s.pat_k.nb
    assert np.diff(s.pat_h.row_ptr).max() <= 128  # b = 4 list plans take Bt rows of <= 128 blocks
    kset = [set(s.pat_k.col_idx[s.pat_k.row_ptr[i]:s.pat_k.row_ptr[i + 1]]) for i in range(nb)]
    hset = [set(s.pat_h.col_idx[s.pat_h.row_ptr[j]:s.pat_h.row_ptr[j + 1]]) for j in range(nb)]
    hits = max(len(kset[i] & hset[j]) for i in range(0, nb, 7) for j in kset[i])
    assert hits > 100
    w = np.linalg.eigvalsh(bm(s.pat_h, s.H).csr().dense())
    lo, hi = float(w[0]) - 0.1, float(w[-1]) + 0.1
    monkeypatch.setenv("CHESS_LISTED_VARIANT", str(variant))
    rng = np.random.default_rng(8)
    coef = rng.standard_normal((2, 50)) / np.arange(1, 51)
    accs, mom = chess_chebyshev(gpu_ctx, dt(s.H), gpat(s.pat_h), lo, hi, gpat(s.pat_k), 50, coef,
                                precision="f32")
    Mt = opl.scaled(bm(s.pat_h, s.H).csr(), lo, hi)
    acc_o, mom_o = ocsr.chebyshev(Mt, bm(s.pat_k).pattern_csr(), 50, coef)
    assert np.max(np.abs(mom - mom_o)) < TOL32 * s.n
    for q in range(2):
        ref = bm(s.pat_k).to_block(acc_o[q])
        assert np.max(np.abs(accs[q].cpu().numpy() - ref)) < TOL32, (variant, q)


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("nq", [1, 2, 4])
def test_b9_chain_kernel_variants(gpu_ctx, monkeypatch, variant, nq):
    # float32 9 x 9 blocks: vector ALU (0), matrix cores (1, 2) and pipelined
    # columns (3, 4; with more than one sum each is read in the column's
    # epilogue), against the oracle
    monkeypatch.setenv("CHESS_LISTED_VARIANT", str(variant))
    s, accs, mom, acc_o, mom_o = chain_case(gpu_ctx, SYS9, 70, "f32", nq=nq)
    assert np.max(np.abs(mom - mom_o)) < TOL32 * s.n
    for q in range(nq):
        ref = bm(s.pat_k).to_block(acc_o[q])
        assert np.max(np.abs(accs[q].cpu().numpy() - ref)) < TOL32, (variant, nq, q)


def test_chain_kernel_variant_out_of_range(gpu_ctx, monkeypatch):
    monkeypatch.setenv("CHESS_LISTED_VARIANT", "27")
    with pytest.raises(ChessError):
        chain_case(gpu_ctx, SYS4, 10, "f32")


@pytest.mark.parametrize("n_pl", [1, 2, 3])
def test_chebyshev_chain_shortest(gpu_ctx, n_pl):
    s, accs, mom, acc_o, mom_o = chain_case(gpu_ctx, SYS4, n_pl, "f64", nq=1)
    assert np.max(np.abs(mom - mom_o)) < 1e-9
    assert np.max(np.abs(accs[0].cpu().numpy() - bm(s.pat_k).to_block(acc_o[0]))) < TOL64


FIX = dict(s_bounds=(0.25, 2.05), bounds=(-1.9, 0.1), n_pl=180, n_pl_s=40)


def oracle_fermi(s, **kw):
    Ko, info = opl.fermi_operator(bm(s.pat_h, s.H), bm(s.pat_h, s.S), bm(s.pat_k), s.n_electrons,
                                  s.kT, **kw)
    return Ko, info


@pytest.mark.parametrize("spec", [SYS4, SYS9])
@pytest.mark.parametrize("precision,tol", [("f64", TOL64), ("f32", TOL32)])
def test_fermi_operator_fixed_parameters(gpu_ctx, spec, precision, tol):
    s = system(*spec, kT=0.02)
    mu = -0.95
    K, info = chess_fermi_operator(gpu_ctx, dt(s.H), gpat(s.pat_h), dt(s.S), gpat(s.pat_h),
                                   gpat(s.pat_k), s.n_electrons, s.kT, precision=precision,
                                   mu=mu, **FIX)
    Ko, oinfo = oracle_fermi(s, s_bounds_=FIX["s_bounds"], n_pl_s=FIX["n_pl_s"],
                             h_bounds=FIX["bounds"], n_pl=FIX["n_pl"], mu=mu)
    assert np.max(np.abs(K.cpu().numpy() - Ko)) < tol
    assert abs(info["tr_ks"] - oinfo["trKS"]) < tol * s.n


@pytest.mark.parametrize("history", [0, 1])
def test_fermi_operator_mu_search(gpu_ctx, history):
    s = system(*SYS4, kT=0.02)
    fx = dict(FIX)
    K, info = chess_fermi_operator(gpu_ctx, dt(s.H), gpat(s.pat_h), dt(s.S), gpat(s.pat_h),
                                   gpat(s.pat_k), s.n_electrons, s.kT, precision="f64",
                                   store_history=history, tol_ne=1e-11, **fx)
    Ko, oinfo = oracle_fermi(s, s_bounds_=fx["s_bounds"], n_pl_s=fx["n_pl_s"],
                             h_bounds=fx["bounds"], n_pl=fx["n_pl"], tol_ne=1e-11)
    assert abs(info["mu"] - oinfo["mu"]) < 1e-9
    assert abs(info["ne_chain"] - s.n_electrons) < 1e-9
    assert np.max(np.abs(K.cpu().numpy() - Ko)) < 1e-8
    assert info["passes"] == (1 if history else 2)


def test_fermi_operator_dense_matches_diagonalisation(gpu_ctx):
    # dense patterns (both cutoffs exceed the box): no truncation, so the result
    # is the exact density kernel up to the polynomial error
    s = system(64, 4, 10.0, 14.0, 0, kT=0.01)
    Hd, Sd = g.to_dense(s.pat_h, s.H), g.to_dense(s.pat_h, s.S)
    Kd, mu, ev = odense.density_kernel(Hd, Sd, s.n_electrons, s.kT)
    K, info = chess_fermi_operator(gpu_ctx, dt(s.H), gpat(s.pat_h), dt(s.S), gpat(s.pat_h),
                                   gpat(s.pat_k), s.n_electrons, s.kT, precision="f64",
                                   s_bounds=(0.299, 2.001), bounds=(ev[0] - 1e-3, ev[-1] + 1e-3),
                                   tol_fit=1e-13, tol_fit_s=1e-13, tol_ne=1e-12)
    assert abs(info["mu"] - mu) < 1e-10
    assert np.max(np.abs(K.cpu().numpy() - g.from_dense(s.pat_k, Kd))) < TOL64
    assert abs(info["tr_ks"] - s.n_electrons) < 1e-9


@pytest.mark.parametrize("precision,tol", [("f64", TOL64), ("f32", TOL32)])
def test_fermi_dirac_fixed_parameters(gpu_ctx, precision, tol):
    # Eq. 9 occupation (smearing = Fermi-Dirac) against the oracle's
    s = system(*SYS4, kT=0.02)
    K, info = chess_fermi_operator(gpu_ctx, dt(s.H), gpat(s.pat_h), dt(s.S), gpat(s.pat_h),
                                   gpat(s.pat_k), s.n_electrons, s.kT, precision=precision,
                                   smearing="fermi_dirac", mu=-0.95, **FIX)
    Ko, oinfo = oracle_fermi(s, smearing="fd", s_bounds_=FIX["s_bounds"], n_pl_s=FIX["n_pl_s"],
                             h_bounds=FIX["bounds"], n_pl=FIX["n_pl"], mu=-0.95)
    assert np.max(np.abs(K.cpu().numpy() - Ko)) < tol
    assert abs(info["tr_ks"] - oinfo["trKS"]) < tol * s.n


def test_fermi_dirac_mu_search(gpu_ctx):
    s = system(*SYS4, kT=0.02)
    K, info = chess_fermi_operator(gpu_ctx, dt(s.H), gpat(s.pat_h), dt(s.S), gpat(s.pat_h),
                                   gpat(s.pat_k), s.n_electrons, s.kT, precision="f64",
                                   smearing="fermi_dirac", tol_ne=1e-11, **FIX)
    Ko, oinfo = oracle_fermi(s, smearing="fd", s_bounds_=FIX["s_bounds"], n_pl_s=FIX["n_pl_s"],
                             h_bounds=FIX["bounds"], n_pl=FIX["n_pl"], tol_ne=1e-11)
    assert abs(info["mu"] - oinfo["mu"]) < 1e-9
    assert np.max(np.abs(K.cpu().numpy() - Ko)) < 1e-8
    assert abs(info["homo"] - oinfo["homo"]) < 1e-8 and abs(info["lumo"] - oinfo["lumo"]) < 1e-8


def test_fermi_dirac_dense_matches_diagonalisation(gpu_ctx):
    # no truncation on dense patterns: the exact Fermi-Dirac density kernel up
    # to the polynomial error, with mu from the library's own search
    s = system(64, 4, 10.0, 14.0, 0, kT=0.03)
    Hd, Sd = g.to_dense(s.pat_h, s.H), g.to_dense(s.pat_h, s.S)
    Kd, mu, ev = odense.density_kernel(Hd, Sd, s.n_electrons, s.kT, smearing="fd")
    K, info = chess_fermi_operator(gpu_ctx, dt(s.H), gpat(s.pat_h), dt(s.S), gpat(s.pat_h),
                                   gpat(s.pat_k), s.n_electrons, s.kT, precision="f64",
                                   smearing="fermi_dirac", s_bounds=(0.299, 2.001),
                                   bounds=(ev[0] - 1e-3, ev[-1] + 1e-3), tol_fit=1e-13,
                                   tol_fit_s=1e-13, tol_ne=1e-12)
    assert abs(info["mu"] - mu) < 1e-10
    assert np.max(np.abs(K.cpu().numpy() - g.from_dense(s.pat_k, Kd))) < TOL64
    assert abs(info["tr_ks"] - s.n_electrons) < 1e-9


@pytest.mark.parametrize("a", [-1.0, -0.5, 0.5])
@pytest.mark.parametrize("spec", [SYS4, SYS9])
@pytest.mark.parametrize("precision,tol", [("f64", TOL64), ("f32", TOL32)])
def test_matrix_power_parity(gpu_ctx, a, spec, precision, tol):
    # S is scaled to the spectrum [0.3, 2.0] by the generator
    s = system(*spec)
    R, info = chess_matrix_power(gpu_ctx, dt(s.S), gpat(s.pat_h), a, gpat(s.pat_k),
                                 precision=precision, s_bounds=(0.25, 2.05), n_pl_s=48)
    assert info["n_pl_s"] == 48
    Ro, _ = opl.matrix_power(bm(s.pat_h, s.S), a, bm(s.pat_k), bounds=(0.25, 2.05), n_pl=48)
    assert np.max(np.abs(R.cpu().numpy() - Ro)) < tol


def test_matrix_power_estimated_bounds(gpu_ctx):
    # bounds estimated on the GPU (Gershgorin upper, Lanczos lower): the result
    # must match the exact power on a dense pattern
    s = system(64, 4, 10.0, 14.0, 0)
    Sd = g.to_dense(s.pat_h, s.S)
    R, info = chess_matrix_power(gpu_ctx, dt(s.S), gpat(s.pat_h), -0.5, gpat(s.pat_k),
                                 precision="f64", tol_fit_s=1e-12)
    assert 0 < info["s_lo"] <= 0.3 and info["s_hi"] >= 2.0
    ref = g.from_dense(s.pat_k, odense.matrix_power(Sd, -0.5))
    assert np.max(np.abs(R.cpu().numpy() - ref)) < 1e-9


def test_eigs_in_interval_parity(gpu_ctx):
    s = system(*SYS4)
    width, n_pl = 3e-3, 1200
    lo, hi = -1.1, -0.9
    ev, info = chess_eigs_in_interval(gpu_ctx, dt(s.H), gpat(s.pat_h), dt(s.S), gpat(s.pat_h), lo,
                                      hi, gpat(s.pat_k), precision="f64", eig_width=width,
                                      n_pl=n_pl, s_bounds=(0.25, 2.05), n_pl_s=40,
                                      bounds=(-1.9, 0.1))
    ref, _ = opl.eigs_in_interval(bm(s.pat_h, s.H), bm(s.pat_h, s.S), bm(s.pat_k), lo, hi,
                                  width=width, s_bounds_=(0.25, 2.05), n_pl_s=40,
                                  h_bounds=(-1.9, 0.1), n_pl=n_pl)
    assert ev.shape == ref.shape and ev.shape[0] > 5
    assert np.max(np.abs(ev - ref)) < 1e-8


def test_eigs_in_interval_parity_b9(gpu_ctx):
    # 9 x 9 blocks: H' of this system lies in [-1.70, -0.30]; a fixed degree
    # and an interval of about ten eigenvalues keep the oracle's bisections short
    s = system(*SYS9)
    lo, hi, width, n_pl = -0.95, -0.93, 3e-3, 1200
    ev, info = chess_eigs_in_interval(gpu_ctx, dt(s.H), gpat(s.pat_h), dt(s.S), gpat(s.pat_h), lo,
                                      hi, gpat(s.pat_k), precision="f64", eig_width=width,
                                      n_pl=n_pl, s_bounds=(0.25, 2.05), n_pl_s=40,
                                      bounds=(-1.9, 0.1))
    print(f"[gpu-parity] b9 eigenvalues: {ev.shape[0]} from the library", flush=True)
    ref, _ = opl.eigs_in_interval(bm(s.pat_h, s.H), bm(s.pat_h, s.S), bm(s.pat_k), lo, hi,
                                  width=width, s_bounds_=(0.25, 2.05), n_pl_s=40,
                                  h_bounds=(-1.9, 0.1), n_pl=n_pl)
    assert ev.shape == ref.shape and ev.shape[0] > 5
    assert np.max(np.abs(ev - ref)) < 1e-8


def test_errors_are_reported(gpu_ctx):
    s = system(*SYS4)
    H, S = dt(s.H), dt(s.S)
    ph, pk = gpat(s.pat_h), gpat(s.pat_k)
    with pytest.raises(ChessError) as e:
        chess_fermi_operator(gpu_ctx, H, ph, S, ph, pk, 10 * s.n, s.kT)
    assert e.value.name == "CHESS_E_ARG"
    # H pattern not inside the kernel pattern: swap the roles
    with pytest.raises(ChessError) as e:
        chess_matrix_power(gpu_ctx, dt(np.zeros((s.pat_k.nnzb, 4, 4)) + 0.01), pk, 1.0, ph)
    assert e.value.name == "CHESS_E_PATTERN"
    # a missing diagonal block
    rp = s.pat_h.row_ptr.copy()
    ci = s.pat_h.col_idx.copy()
    row0 = ci[rp[0]:rp[1]]
    keep = np.ones(ci.shape[0], bool)
    keep[rp[0] + int(np.nonzero(row0 == 0)[0][0])] = False
    ci2 = ci[keep]
    rp2 = rp.copy()
    rp2[1:] -= 1
    bad = BlockPattern.from_host(4, rp2, ci2)
    with pytest.raises(ChessError) as e:
        chess_matrix_power(gpu_ctx, dt(s.S[keep]), bad, 1.0, pk)
    assert e.value.name == "CHESS_E_PATTERN"
    # S indefinite with a non-integer power
    Sneg = s.S.copy()
    Sneg[g.positions_in_pattern(s.pat_h, np.arange(s.pat_h.nb), np.arange(s.pat_h.nb))] -= 3 * np.eye(4)
    with pytest.raises(ChessError) as e:
        chess_matrix_power(gpu_ctx, dt(Sneg), ph, -0.5, pk, precision="f64")
    assert e.value.name == "CHESS_E_NOT_SPD"
    with pytest.raises(ChessError) as e:
        chess_eigs_in_interval(gpu_ctx, H, ph, S, ph, -1.1, -0.9, pk, capacity=2, precision="f64",
                               n_pl=200, s_bounds=(0.25, 2.05), n_pl_s=40, bounds=(-1.9, 0.1))
    assert e.value.name == "CHESS_E_CAPACITY"


@pytest.mark.parametrize("rows", [1, 2])
@pytest.mark.parametrize("precision,tol", [("f64", TOL64), ("f32", TOL32)])
def test_chain_tile_heights(gpu_ctx, monkeypatch, rows, precision, tol):
    # b = 4 plans with tiles of other heights than 4 (the tile tuner's
    # alternatives; the output-stationary kernel), two sums, against the oracle
    monkeypatch.setenv("CHESS_TILE_ROWS", str(rows))
    s, accs, mom, acc_o, mom_o = chain_case(gpu_ctx, SYSL, 70, precision, nq=2)
    assert np.max(np.abs(mom - mom_o)) < tol * s.n
    for q in range(2):
        ref = bm(s.pat_k).to_block(acc_o[q])
        assert np.max(np.abs(accs[q].cpu().numpy() - ref)) < tol, (rows, precision, q)


def test_fermi_operator_reports_its_tile_height(gpu_ctx, monkeypatch):
    s = system(*SYS4)
    common = dict(precision="f32", s_bounds=(0.25, 2.05), n_pl_s=40, bounds=(-1.9, 0.1), n_pl=120,
                  mu=-0.95)
    K4, i4 = chess_fermi_operator(gpu_ctx, dt(s.H), gpat(s.pat_h), dt(s.S), gpat(s.pat_h),
                                  gpat(s.pat_k), s.n_electrons, 0.02, **common)
    assert i4["tile_rows"] in (2, 4)
    monkeypatch.setenv("CHESS_TILE_ROWS", "2")
    K2, i2 = chess_fermi_operator(gpu_ctx, dt(s.H), gpat(s.pat_h), dt(s.S), gpat(s.pat_h),
                                  gpat(s.pat_k), s.n_electrons, 0.02, **common)
    assert i2["tile_rows"] == 2 and 24 <= i2["kernel_variant"] <= 26
    assert np.max(np.abs(K2.cpu().numpy() - K4.cpu().numpy())) < 1e-5
    monkeypatch.setenv("CHESS_TILE_ROWS", "3")  # no kernel is built for 3-row tiles
    with pytest.raises(ChessError) as e:
        chess_fermi_operator(gpu_ctx, dt(s.H), gpat(s.pat_h), dt(s.S), gpat(s.pat_h),
                             gpat(s.pat_k), s.n_electrons, 0.02, **common)
    assert e.value.name == "CHESS_E_ARG"


@pytest.mark.parametrize("spec", ["SYS4", "SYS9"])
@pytest.mark.parametrize("n_pl", [5, 61, 70])
@pytest.mark.parametrize("precision,tol", [("f64", TOL64), ("f32", TOL32)])
def test_moments_only_chain_runs_half(gpu_ctx, monkeypatch, spec, n_pl, precision, tol):
    # a moments-only chain computes T_m up to m = n_pl / 2 and the other
    # moments from <T_m, T_m> and <T_{m+1}, T_m> (product rule of Chebyshev
    # polynomials, exact for the truncated chain); against the oracle's
    # directly computed moments and against the library's full chain
    sp = {"SYS4": SYS4, "SYS9": SYS9}[spec]
    s = system(*sp)
    e0, e1 = g.extreme_eigenvalues(s.pat_h, s.H)
    lo, hi = e0 - 0.02 * (e1 - e0), e1 + 0.02 * (e1 - e0)
    _, mom = chess_chebyshev(gpu_ctx, dt(s.H), gpat(s.pat_h), lo, hi, gpat(s.pat_k), n_pl,
                             precision=precision)
    Mt = opl.scaled(bm(s.pat_h, s.H).csr(), lo, hi)
    _, mom_o = ocsr.chebyshev(Mt, bm(s.pat_k).pattern_csr(), n_pl, None)
    assert np.max(np.abs(mom - mom_o)) < tol * s.n, (spec, n_pl, precision)
    monkeypatch.setenv("CHESS_FULL_MOMENTS", "1")
    _, mom_f = chess_chebyshev(gpu_ctx, dt(s.H), gpat(s.pat_h), lo, hi, gpat(s.pat_k), n_pl,
                               precision=precision)
    assert np.max(np.abs(mom - mom_f)) < tol * s.n


@pytest.mark.parametrize("precision,variant,tol", [("f32", 24, TOL32), ("f32", 20, TOL32),
                                                   ("f64", 12, TOL64), ("f64", 2, TOL64)])
def test_moments_only_chain_fused_and_separate_dots(gpu_ctx, monkeypatch, precision, variant, tol):
    # the output-stationary kernel adds the Frobenius products in its
    # epilogue (24, 12); the other kernels leave them to k_dot_pair (20, 2)
    monkeypatch.setenv("CHESS_LISTED_VARIANT", str(variant))
    s = system(*SYSL)
    e0, e1 = g.extreme_eigenvalues(s.pat_h, s.H)
    lo, hi = e0 - 0.02 * (e1 - e0), e1 + 0.02 * (e1 - e0)
    for n_pl in (64, 71):
        _, mom = chess_chebyshev(gpu_ctx, dt(s.H), gpat(s.pat_h), lo, hi, gpat(s.pat_k), n_pl,
                                 precision=precision)
        Mt = opl.scaled(bm(s.pat_h, s.H).csr(), lo, hi)
        _, mom_o = ocsr.chebyshev(Mt, bm(s.pat_k).pattern_csr(), n_pl, None)
        assert np.max(np.abs(mom - mom_o)) < tol * s.n, (precision, variant, n_pl)
