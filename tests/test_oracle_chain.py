"""Pins of the oracle's matrix part (masked product, truncated chain) and of
the whole oracle pipeline against dense definitions and invariants.  CPU only."""
import numpy as np
import scipy.linalg
import scipy.sparse as sp

from oracle import chebyshev as cb
from oracle import dense
from oracle import pipeline as pl
from oracle.csr import Csr, chebyshev, masked_spgemm
from workloads import generator as g


def random_pattern(n, density, rng, sym=True):
    M = sp.random(n, n, density=density, random_state=np.random.RandomState(rng.integers(1 << 30)))
    M = (M + M.T) if sym else M
    M = M + sp.eye(n)
    M = sp.csr_matrix(M)
    M.sort_indices()
    return Csr(n, M.indptr, M.indices)


def test_masked_product_is_exact_on_integers():
    # Integer-valued entries make every sum exact in float64, so the result
    # equals the dense product restricted to the pattern bit for bit.
    rng = np.random.default_rng(0)
    n = 70
    A = random_pattern(n, 0.08, rng, sym=False)
    B = random_pattern(n, 0.1, rng, sym=False)
    C = random_pattern(n, 0.15, rng)
    A.v = rng.integers(-9, 10, A.nnz).astype(np.float64)
    B.v = rng.integers(-9, 10, B.nnz).astype(np.float64)
    out = masked_spgemm(A, B, C)
    ref = A.dense() @ B.dense()
    assert np.array_equal(out, C.values_from_dense(ref))


def test_chain_on_a_diagonal_matrix():
    # Diagonal M~: T_k = diag(cos(k arccos d)), exactly the scalar recursion.
    n = 50
    d = np.linspace(-0.97, 0.99, n)
    M = Csr(n, np.arange(n + 1), np.arange(n), d)
    K = random_pattern(n, 0.1, np.random.default_rng(1))
    n_pl = 30
    coef = np.random.default_rng(2).standard_normal((2, n_pl))
    acc, mom = chebyshev(M, K, n_pl, coef)
    th = np.arccos(d)
    Tk = np.cos(np.outer(np.arange(n_pl), th))  # [k, i]
    assert np.max(np.abs(mom - Tk.sum(axis=1))) < 1e-12
    for q in range(2):
        diag_ref = 0.5 * coef[q, 0] + coef[q, 1:] @ Tk[1:]
        D = K.with_values(acc[q]).dense()
        assert np.max(np.abs(np.diag(D) - diag_ref)) < 1e-12
        assert np.max(np.abs(D - np.diag(np.diag(D)))) == 0.0


def test_chain_on_a_dense_pattern_is_the_matrix_function():
    # With no truncation, T_k = V cos(k arccos L) V^T.
    rng = np.random.default_rng(3)
    n = 40
    A = rng.standard_normal((n, n))
    A = A + A.T
    w, V = np.linalg.eigh(A)
    A = A / (1.05 * np.max(np.abs(w)))
    w, V = np.linalg.eigh(A)
    full = Csr.from_scipy(sp.csr_matrix(np.ones((n, n))))
    M = full.with_values(full.values_from_dense(A))
    n_pl = 25
    coef = rng.standard_normal((1, n_pl))
    acc, mom = chebyshev(M, full, n_pl, coef)
    th = np.arccos(w)
    ref = V @ np.diag(0.5 * coef[0, 0] + np.cos(np.outer(np.arange(1, n_pl), th)).T @ coef[0, 1:]) @ V.T
    assert np.max(np.abs(full.with_values(acc[0]).dense() - ref)) < 1e-12
    assert np.max(np.abs(mom - np.cos(np.outer(np.arange(n_pl), th)).sum(axis=1))) < 1e-11


def test_chain_columns_follow_the_recursion_independently():
    # Left multiplication: column j of T_{k+1} is P_K(:, j) o (2 M~ t_k) - t_{k-1}
    # with sparse matrix-vector products only (Sec. "Expansion in Chebyshev
    # polynomials": columns are independent).
    rng = np.random.default_rng(4)
    n = 60
    Mp = random_pattern(n, 0.05, rng)
    K = random_pattern(n, 0.12, rng)
    Kd = (K.with_values(np.ones(K.nnz)).dense() != 0)
    Md = Mp.with_values(rng.standard_normal(Mp.nnz)).dense()
    Md = 0.5 * (Md + Md.T)
    Md = Md * (Mp.with_values(np.ones(Mp.nnz)).dense() != 0)
    Md /= 1.1 * np.max(np.abs(np.linalg.eigvalsh(Md)))
    Ms = sp.csr_matrix(Md)
    M = Csr.from_scipy(Ms)
    # make sure P_M within P_K
    K = Csr.from_scipy(sp.csr_matrix((Kd | (Md != 0)).astype(float)))
    Kd = K.with_values(np.ones(K.nnz)).dense() != 0
    n_pl = 12
    coef = np.zeros((1, n_pl))
    coef[0, -1] = 1.0  # acc = T_{n_pl-1}
    acc, _ = chebyshev(M, K, n_pl, coef)
    T_last = K.with_values(acc[0]).dense()
    for j in (0, 17, 59):
        e = np.zeros(n)
        e[j] = 1.0
        tm, t = e, Kd[:, j] * (Ms @ e)
        for _ in range(2, n_pl):
            tm, t = t, Kd[:, j] * (2 * (Ms @ t)) - tm
        assert np.max(np.abs(T_last[:, j] - t)) < 1e-12


def test_block_diagonal_pattern_gives_independent_block_functions():
    # With P_K = block diagonal, the chain is the matrix function of each
    # diagonal block of M~ separately.
    b, nb = 4, 6
    rng = np.random.default_rng(5)
    rp = np.arange(nb + 1)
    ci = np.arange(nb)
    blocks = rng.standard_normal((nb, b, b))
    blocks = 0.5 * (blocks + np.transpose(blocks, (0, 2, 1)))
    blocks /= 1.2 * np.max(np.abs(np.linalg.eigvalsh(blocks)))
    M = pl.BlockMat(nb, b, rp, ci, blocks)
    Mc = M.csr()
    n_pl = 20
    coef = rng.standard_normal((1, n_pl))
    acc, _ = chebyshev(Mc, M.pattern_csr(), n_pl, coef)
    out = M.to_block(acc[0])
    for i in range(nb):
        w, V = np.linalg.eigh(blocks[i])
        fv = 0.5 * coef[0, 0] + np.cos(np.outer(np.arange(1, n_pl), np.arccos(w))).T @ coef[0, 1:]
        assert np.max(np.abs(out[i] - V @ np.diag(fv) @ V.T)) < 1e-12


def small_dense_system(n_atoms=16, seed=3, kT=0.02):
    s = g.make_system(n_atoms, 4, 10.0, 14.0, seed=seed, kT=kT)
    H = pl.BlockMat(s.pat_h.nb, 4, s.pat_h.row_ptr, s.pat_h.col_idx, s.H)
    S = pl.BlockMat(s.pat_h.nb, 4, s.pat_h.row_ptr, s.pat_h.col_idx, s.S)
    K = pl.BlockMat(s.pat_k.nb, 4, s.pat_k.row_ptr, s.pat_k.col_idx)
    return s, H, S, K


def test_fermi_operator_matches_diagonalisation_on_dense_pattern():
    s, H, S, K = small_dense_system()
    Hd, Sd = g.to_dense(s.pat_h, s.H), g.to_dense(s.pat_h, s.S)
    Kd, mu, ev = dense.density_kernel(Hd, Sd, s.n_electrons, s.kT)
    Kv, info = pl.fermi_operator(H, S, K, s.n_electrons, s.kT, s_bounds_=(0.29, 2.01),
                                 h_bounds=(ev[0] - 0.01, ev[-1] + 0.01), tol_fit=1e-13,
                                 tol_fit_s=1e-13, tol_ne=1e-12)
    assert abs(info["mu"] - mu) < 1e-10
    assert np.max(np.abs(Kv - g.from_dense(s.pat_k, Kd))) < 1e-10
    assert abs(info["trKS"] - s.n_electrons) < 1e-9


def test_fermi_dirac_variant_matches_diagonalisation():
    s, H, S, K = small_dense_system(seed=4, kT=0.03)
    Hd, Sd = g.to_dense(s.pat_h, s.H), g.to_dense(s.pat_h, s.S)
    Kd, mu, ev = dense.density_kernel(Hd, Sd, s.n_electrons, s.kT, smearing="fd")
    Kv, info = pl.fermi_operator(H, S, K, s.n_electrons, s.kT, smearing="fd",
                                 s_bounds_=(0.29, 2.01), h_bounds=(ev[0] - 0.01, ev[-1] + 0.01),
                                 tol_fit=1e-12, tol_fit_s=1e-13, mu=mu)
    assert np.max(np.abs(Kv - g.from_dense(s.pat_k, Kd))) < 1e-9


def test_idempotency_for_a_gapped_spectrum():
    # Designed spectrum with a gap at mu and kT well below the gap: K S K = K
    # up to max f(1 - f) (Eq. 10 with occupations in {0, 1}).
    rng = np.random.default_rng(6)
    n, nocc = 48, 20
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([rng.uniform(-1.0, -0.6, nocc), rng.uniform(-0.2, 0.4, n - nocc)])
    Sd = Q @ np.diag(rng.uniform(0.5, 1.5, n)) @ Q.T
    Sh = scipy.linalg.sqrtm(Sd).real
    Hd = Sh @ (Q @ np.diag(lam) @ Q.T) @ Sh  # generalized eigenvalues = lam
    Hd = 0.5 * (Hd + Hd.T)
    b = 4
    full = g.BlockPattern(nb=n // b, b=b, row_ptr=np.arange(0, (n // b) ** 2 + 1, n // b),
                          col_idx=np.tile(np.arange(n // b), n // b).astype(np.int32))
    H = pl.BlockMat(full.nb, b, full.row_ptr, full.col_idx, g.from_dense(full, Hd))
    S = pl.BlockMat(full.nb, b, full.row_ptr, full.col_idx, g.from_dense(full, Sd))
    P = pl.BlockMat(full.nb, b, full.row_ptr, full.col_idx)
    ws = np.linalg.eigvalsh(Sd)
    kT = 0.02
    Kv, info = pl.fermi_operator(H, S, P, float(nocc), kT, s_bounds_=(ws[0] * 0.99, ws[-1] * 1.01),
                                 h_bounds=(-1.05, 0.45), tol_fit=1e-12, tol_fit_s=1e-13)
    Kd = g.to_dense(full, Kv)
    f = cb.occ_erfc(lam, info["mu"], kT)
    bound = np.max(f * (1 - f)) * 1.01 + 1e-9
    assert np.max(np.abs(Kd @ Sd @ Kd - Kd)) <= bound * np.max(np.abs(np.linalg.inv(Sd))) + 1e-9
    assert abs(info["trKS"] - nocc) < 1e-6


def test_matrix_powers_dense_and_inverse_identity():
    s, H, S, K = small_dense_system(seed=5)
    Sd = g.to_dense(s.pat_h, s.S)
    for a in (-1.0, -0.5, 0.5):
        v, info = pl.matrix_power(S, a, K, bounds=(0.29, 2.01), tol_fit=1e-13)
        ref = g.from_dense(s.pat_k, dense.matrix_power(Sd, a))
        assert np.max(np.abs(v - ref)) < 1e-11, a
    # S^a S^-a = I (Eq. 12's identity test on a dense pattern)
    vp, _ = pl.matrix_power(S, 0.5, K, bounds=(0.29, 2.01), tol_fit=1e-13)
    vm, _ = pl.matrix_power(S, -0.5, K, bounds=(0.29, 2.01), tol_fit=1e-13)
    prod = g.to_dense(s.pat_k, vp) @ g.to_dense(s.pat_k, vm)
    assert np.max(np.abs(prod - np.eye(s.n))) < 1e-11


def test_sparse_inverse_error_measures_are_small():
    # Sparse S with a buffer pattern: Eq. 13 against the cropped exact inverse
    # and Eq. 12 for S^-1 applied twice (values reported by the paper's accuracy
    # section only as plots; here they must simply be small).
    prev = None
    for r_k in (6.0, 7.0):
        s = g.make_system(200, 4, 4.5, r_k, seed=11)
        S = pl.BlockMat(s.pat_h.nb, 4, s.pat_h.row_ptr, s.pat_h.col_idx, s.S)
        K = pl.BlockMat(s.pat_k.nb, 4, s.pat_k.row_ptr, s.pat_k.col_idx)
        inv, info = pl.matrix_power(S, -1.0, K, bounds=(0.29, 2.01), tol_fit=1e-12)
        Sd = g.to_dense(s.pat_h, s.S)
        exact = g.from_dense(s.pat_k, np.linalg.inv(Sd))
        w13 = dense.w_sparse(inv, exact)
        assert w13 < 1e-5
        if prev is not None:
            assert w13 < prev  # a larger buffer region absorbs more of the decay
        prev = w13
        Kinv = pl.BlockMat(s.pat_k.nb, 4, s.pat_k.row_ptr, s.pat_k.col_idx, inv)
        back, _ = pl.matrix_power(Kinv, -1.0, K, bounds=(0.4, 4.0), tol_fit=1e-12)
        w12 = dense.w_inverse_identity(back, g.from_dense(s.pat_k, Sd))
        assert w12 < 1e-5


def test_eigenvalues_in_interval_against_diagonalisation():
    s, H, S, K = small_dense_system(seed=8)
    Hd, Sd = g.to_dense(s.pat_h, s.H), g.to_dense(s.pat_h, s.S)
    ev = scipy.linalg.eigh(Hd, Sd, eigvals_only=True)
    lo, hi = ev[20] - 1e-3, ev[40] + 1e-3
    width = 3e-3
    # n_pl = 1184 is what Eq. 7 gives for this width at tol_fit 1e-7
    got, info = pl.eigs_in_interval(H, S, K, lo, hi, width=width, s_bounds_=(0.29, 2.01),
                                    h_bounds=(ev[0] - 0.01, ev[-1] + 0.01), n_pl=1184)
    ref = ev[(ev >= lo) & (ev <= hi)]
    assert got.shape == ref.shape
    gaps = np.minimum(np.diff(np.concatenate([[-1e9], ref])), np.diff(np.concatenate([ref, [1e9]])))
    sep = gaps > 3 * width  # well separated eigenvalues are found to high accuracy
    assert sep.sum() >= 8
    assert np.max(np.abs(got - ref)[sep]) < 0.01 * width
    assert np.max(np.abs(got - ref)) < 0.5 * width


def test_generator_patterns_match_brute_force():
    s = g.make_system(1600, 4, 4.57, 5.99, seed=2)  # k-d tree path
    for pat, rc in ((s.pat_h, 4.57), (s.pat_k, 5.99)):
        ref = g.brute_force_pattern(s.pos, s.box, rc, 4)
        assert np.array_equal(pat.row_ptr, ref.row_ptr)
        assert np.array_equal(pat.col_idx, ref.col_idx)
    assert np.all(np.isin(np.arange(1), [0]))


def test_generator_matrices_are_symmetric_with_the_stated_spectrum():
    s = g.make_system(64, 4, 10.0, 14.0, seed=0)
    Sd, Hd = g.to_dense(s.pat_h, s.S), g.to_dense(s.pat_h, s.H)
    assert np.array_equal(Sd, Sd.T) and np.array_equal(Hd, Hd.T)
    w = np.linalg.eigvalsh(Sd)
    assert abs(w[0] - 0.3) < 1e-12 and abs(w[-1] - 2.0) < 1e-12
    assert s.pat_h.nnzb == 64 * 64  # both cutoffs exceed the box: dense
