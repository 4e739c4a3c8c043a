"""Seeded synthetic systems that stand in for the paper's BigDFT matrices.

Input infrastructure only: this module draws atoms, builds block sparsity
patterns from distance cutoffs and fills the overlap S and Hamiltonian H with
random values.  It contains none of the method's arithmetic (no Chebyshev
expansion, no bounds, no chemical potential), so both the oracle and the HIP
path may take their inputs from it.

Structure follows the paper's benchmark setup (Sec. "Performance", first
paragraph): sparsity patterns from geometric cutoffs, nested so that S and H
share a sparser pattern and the kernel/inverse pattern is a superset with a
buffer region; values are random with the spectral properties the tests need.

Readings (all choices the paper leaves open):
  * positions: random sequential placement in a periodic cube at a density of
    0.1 atoms/bohr^3 with a minimum image distance of 1.8 bohr, then Morton
    order (this changes only memory locality, not the mathematics);
  * a block pair (A, B) is in a pattern iff dx^2+dy^2+dz^2 < rc^2 in float64,
    with the minimum image dx -= L*rint(dx/L), evaluated in that order;
  * S_AA = I_b, S_AB = exp(-r^2/8) (I_b + 0.05 G) with G iid N(0,1) per
    unordered pair, S_BA = S_AB^T; then S <- a S + c I maps its extreme
    eigenvalues onto [0.3, 2.0] exactly (dense eigvalsh up to 9000 rows,
    otherwise implicitly restarted Lanczos to a relative 1e-8);
  * H_AA = diag(U[-0.7, -0.3]) per basis function, H_AB = -0.3 exp(-r/2)
    (I_b + 0.05 G'), mirrored;
  * S and H both live on the pattern with cutoff r_H; the kernel pattern uses
    r_K >= r_H.

Storage: block CSR, uniform block edge b, row_ptr int64 [nb+1], col_idx int32
[nnzb] strictly increasing per row with the diagonal present, values float64
[nnzb, b, b] with each block row-major.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg
import scipy.spatial

RHO = 0.1
DMIN = 1.8


@dataclass
class BlockPattern:
    nb: int
    b: int
    row_ptr: np.ndarray  # int64 [nb+1]
    col_idx: np.ndarray  # int32 [nnzb]

    @property
    def nnzb(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def n(self) -> int:
        return self.nb * self.b

    def rows(self) -> np.ndarray:
        return np.repeat(np.arange(self.nb, dtype=np.int64), np.diff(self.row_ptr))


@dataclass
class System:
    pos: np.ndarray
    box: float
    b: int
    pat_h: BlockPattern
    pat_k: BlockPattern
    S: np.ndarray  # float64 [nnzb_h, b, b]
    H: np.ndarray  # float64 [nnzb_h, b, b]
    n_electrons: float
    kT: float
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.pat_h.n


# ----------------------------------------------------------------------------
# positions
# ----------------------------------------------------------------------------

def place_atoms(n_atoms: int, rng: np.random.Generator, rho: float = RHO,
                dmin: float = DMIN) -> tuple[np.ndarray, float]:
    """Random sequential placement in a periodic cube of side (n/rho)^(1/3)."""
    L = (n_atoms / rho) ** (1.0 / 3.0)
    ncell = max(1, int(math.floor(L / dmin)))
    cs = L / ncell
    cells: dict[tuple[int, int, int], list[tuple[float, float, float]]] = {}
    out: list[tuple[float, float, float]] = []
    d2min = dmin * dmin
    offs = [(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)]
    if ncell < 3:
        offs = None  # small box: check everything
    batch = rng.random((4096, 3)) * L
    bi = 0
    attempts = 0
    while len(out) < n_atoms:
        if bi == batch.shape[0]:
            batch = rng.random((4096, 3)) * L
            bi = 0
        x, y, z = float(batch[bi, 0]), float(batch[bi, 1]), float(batch[bi, 2])
        bi += 1
        attempts += 1
        if attempts > 200 * n_atoms + 100000:
            raise RuntimeError("random sequential placement did not finish")
        ok = True
        if offs is None:
            cand = out
        else:
            cx, cy, cz = int(x / cs) % ncell, int(y / cs) % ncell, int(z / cs) % ncell
            cand = []
            for (i, j, k) in offs:
                cand.extend(cells.get(((cx + i) % ncell, (cy + j) % ncell, (cz + k) % ncell), ()))
        for (px, py, pz) in cand:
            dx = x - px
            dx -= L * round(dx / L)
            dy = y - py
            dy -= L * round(dy / L)
            dz = z - pz
            dz -= L * round(dz / L)
            if dx * dx + dy * dy + dz * dz < d2min:
                ok = False
                break
        if ok:
            out.append((x, y, z))
            if offs is not None:
                cells.setdefault((int(x / cs) % ncell, int(y / cs) % ncell, int(z / cs) % ncell), []).append((x, y, z))
    return np.asarray(out, dtype=np.float64), L


def morton_order(pos: np.ndarray, L: float, bits: int = 10) -> np.ndarray:
    """Permutation sorting atoms by their 3-D Morton (Z-order) code."""
    q = np.clip(np.floor(pos / L * (1 << bits)).astype(np.int64), 0, (1 << bits) - 1)
    code = np.zeros(pos.shape[0], dtype=np.int64)
    for bit in range(bits):
        for d in range(3):
            code |= ((q[:, d] >> bit) & 1) << (3 * bit + d)
    return np.argsort(code, kind="stable")


# ----------------------------------------------------------------------------
# patterns
# ----------------------------------------------------------------------------

def _pair_d2(pos: np.ndarray, L: float, i: np.ndarray, j: np.ndarray) -> np.ndarray:
    d = pos[i] - pos[j]
    d = d - L * np.rint(d / L)
    return d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]


def neighbour_pairs(pos: np.ndarray, L: float, rc: float) -> tuple[np.ndarray, np.ndarray]:
    """All ordered pairs (i, j), i != j, with min-image distance^2 < rc^2.

    Candidates come from a periodic k-d tree with a slightly larger radius; the
    inclusion decision is always the float64 formula stated in the module doc.
    """
    n = pos.shape[0]
    if n <= 1500:
        i, j = np.triu_indices(n, k=1)
    else:
        tree = scipy.spatial.cKDTree(np.mod(pos, L), boxsize=L)
        pr = tree.query_pairs(rc * (1 + 1e-9) + 1e-9, output_type="ndarray")
        i, j = pr[:, 0].astype(np.int64), pr[:, 1].astype(np.int64)
    keep = _pair_d2(pos, L, i, j) < rc * rc
    i, j = i[keep], j[keep]
    ii = np.concatenate([i, j])
    jj = np.concatenate([j, i])
    return ii, jj


def pattern_from_pairs(nb: int, b: int, ii: np.ndarray, jj: np.ndarray) -> BlockPattern:
    """Block CSR pattern from off-diagonal pairs plus the full diagonal."""
    d = np.arange(nb, dtype=np.int64)
    r = np.concatenate([ii.astype(np.int64), d])
    c = np.concatenate([jj.astype(np.int64), d])
    key = np.unique(r * nb + c)
    r = key // nb
    c = key % nb
    row_ptr = np.zeros(nb + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return BlockPattern(nb=nb, b=b, row_ptr=row_ptr, col_idx=c.astype(np.int32))


def brute_force_pattern(pos: np.ndarray, L: float, rc: float, b: int) -> BlockPattern:
    """O(N^2) reference pattern (for tests of the k-d tree path)."""
    n = pos.shape[0]
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    off = i != j
    i, j = i[off], j[off]
    keep = _pair_d2(pos, L, i, j) < rc * rc
    return pattern_from_pairs(n, b, i[keep], j[keep])


# ----------------------------------------------------------------------------
# values
# ----------------------------------------------------------------------------

def positions_in_pattern(pat: BlockPattern, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """Index of block (rows[k], cols[k]) in the pattern's value array (-1 if absent)."""
    key_pat = pat.rows() * pat.nb + pat.col_idx.astype(np.int64)
    key = rows.astype(np.int64) * pat.nb + cols.astype(np.int64)
    p = np.searchsorted(key_pat, key)
    p = np.clip(p, 0, key_pat.shape[0] - 1)
    ok = key_pat[p] == key
    return np.where(ok, p, -1)


def to_dense(pat: BlockPattern, val: np.ndarray) -> np.ndarray:
    b = pat.b
    out = np.zeros((pat.nb, b, pat.nb, b), dtype=val.dtype)
    r = pat.rows()
    out[r, :, pat.col_idx, :] = val
    return out.reshape(pat.n, pat.n)


def from_dense(pat: BlockPattern, M: np.ndarray) -> np.ndarray:
    b = pat.b
    M4 = M.reshape(pat.nb, b, pat.nb, b)
    return np.ascontiguousarray(M4[pat.rows(), :, pat.col_idx, :])


def to_scipy(pat: BlockPattern, val: np.ndarray) -> scipy.sparse.csr_matrix:
    return scipy.sparse.bsr_matrix((val, pat.col_idx, pat.row_ptr),
                                   shape=(pat.n, pat.n)).tocsr()


def _symmetric_block_values(pat: BlockPattern, pos: np.ndarray, L: float,
                            gfun, diag_blocks: np.ndarray, noise: float,
                            rng: np.random.Generator) -> np.ndarray:
    b = pat.b
    rows = pat.rows()
    cols = pat.col_idx.astype(np.int64)
    upper = rows < cols
    iu, ju = rows[upper], cols[upper]
    r = np.sqrt(_pair_d2(pos, L, iu, ju))
    G = rng.standard_normal((iu.shape[0], b, b))
    blk = gfun(r)[:, None, None] * (np.eye(b)[None] + noise * G)
    val = np.zeros((pat.nnzb, b, b))
    val[np.nonzero(upper)[0]] = blk
    lower_pos = positions_in_pattern(pat, ju, iu)
    val[lower_pos] = np.transpose(blk, (0, 2, 1))
    diag_pos = positions_in_pattern(pat, np.arange(pat.nb), np.arange(pat.nb))
    val[diag_pos] = diag_blocks
    return val


def extreme_eigenvalues(pat: BlockPattern, val: np.ndarray) -> tuple[float, float]:
    if pat.n <= 9000:
        w = scipy.linalg.eigvalsh(to_dense(pat, val))
        return float(w[0]), float(w[-1])
    A = to_scipy(pat, val)
    lo = scipy.sparse.linalg.eigsh(A, k=1, which="SA", tol=1e-8, ncv=64, return_eigenvectors=False)[0]
    hi = scipy.sparse.linalg.eigsh(A, k=1, which="LA", tol=1e-8, ncv=64, return_eigenvectors=False)[0]
    return float(lo), float(hi)


def make_system(n_atoms: int, b: int, r_h: float, r_k: float, seed: int,
                kT: float = 0.01, filling: float = 0.5,
                s_range: tuple[float, float] = (0.3, 2.0),
                onsite: tuple[float, float] = (-0.7, -0.3),
                hop: float = 0.3, noise: float = 0.05,
                morton: bool = True) -> System:
    """Draw one system.  Draw order: positions, S noise, onsite, H noise."""
    rng = np.random.default_rng(seed)
    pos, L = place_atoms(n_atoms, rng)
    if morton:
        pos = pos[morton_order(pos, L)]
    ih, jh = neighbour_pairs(pos, L, r_h)
    ik, jk = neighbour_pairs(pos, L, r_k)
    pat_h = pattern_from_pairs(n_atoms, b, ih, jh)
    pat_k = pattern_from_pairs(n_atoms, b, ik, jk)
    eye = np.broadcast_to(np.eye(b), (n_atoms, b, b)).copy()
    S = _symmetric_block_values(pat_h, pos, L, lambda r: np.exp(-r * r / 8.0), eye, noise, rng)
    lo, hi = extreme_eigenvalues(pat_h, S)
    a = (s_range[1] - s_range[0]) / (hi - lo)
    c = s_range[0] - a * lo
    S *= a
    diag_pos = positions_in_pattern(pat_h, np.arange(n_atoms), np.arange(n_atoms))
    S[diag_pos] += c * np.eye(b)[None]
    ons = rng.uniform(onsite[0], onsite[1], size=(n_atoms, b))
    dblk = np.zeros((n_atoms, b, b))
    dblk[:, np.arange(b), np.arange(b)] = ons
    H = _symmetric_block_values(pat_h, pos, L, lambda r: -hop * np.exp(-r / 2.0), dblk, noise, rng)
    n = n_atoms * b
    return System(pos=pos, box=L, b=b, pat_h=pat_h, pat_k=pat_k, S=S, H=H,
                  n_electrons=float(round(filling * n)), kT=kT,
                  meta=dict(n_atoms=n_atoms, r_h=r_h, r_k=r_k, seed=seed))


# ----------------------------------------------------------------------------
# named workloads (sizes of the paper-scale stand-ins)
# ----------------------------------------------------------------------------

CONFIGS = {
    # 64 atoms x 4 -> 256 rows; both cutoffs exceed the box diagonal: dense.
    "dense256": dict(n_atoms=64, b=4, r_h=10.0, r_k=14.0, seed=0, kT=0.01),
    # 1000 atoms x 9 -> 9000 rows; H pattern ~4 %, kernel pattern ~9 %.
    "prec9000": dict(n_atoms=1000, b=9, r_h=4.57, r_k=5.99, seed=1, kT=0.005),
    # 20000 atoms x 4 -> 80000 rows; kernel pattern ~1 % (~64 M values).
    "large80k": dict(n_atoms=20000, b=4, r_h=5.59, r_k=7.82, seed=5, kT=0.003),
    # 2250 atoms x 4 -> 9000 rows with the cutoffs of prec9000 (the same
    # neighbours per atom): the 4 x 4-block stand-in of the precision study,
    # for the bfloat16 operand forms, which need b = 4.
    "prec9000b4": dict(n_atoms=2250, b=4, r_h=4.57, r_k=5.99, seed=1, kT=0.005),
}


# Systems of the learned-predictor data set: physical knobs drawn per seed
# (train seeds 40000 + i, held-out seeds 50000 + i).  Atom counts are
# log-uniform in [n_min, n_max]; b is 4 or 9 with probability 1/2; onsite
# energies are spread +-0.2 Ha around a mean drawn from [-0.8, -0.2]; the
# hopping scale is drawn from [0.2, 0.4]; kT is log-uniform in [0.002, 0.02];
# the filling N_e / n is drawn from [0.25, 0.75]; cutoffs of the 9000-row
# workload (4.57 / 5.99 bohr).
PREDICTOR_TRAIN_SEED0, PREDICTOR_TEST_SEED0 = 40000, 50000


def predictor_system(seed: int, n_min: int = 500, n_max: int = 3000) -> System:
    rng = np.random.default_rng(seed)
    n_atoms = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
    b = 4 if rng.uniform() < 0.5 else 9
    m = rng.uniform(-0.8, -0.2)
    hop = rng.uniform(0.2, 0.4)
    kT = float(np.exp(rng.uniform(np.log(0.002), np.log(0.02))))
    filling = rng.uniform(0.25, 0.75)
    return make_system(n_atoms, b, 4.57, 5.99, seed=seed, kT=kT, filling=filling,
                       onsite=(m - 0.2, m + 0.2), hop=hop)


# The batched workload: 48 systems, atom counts log-uniform in [200, 4000],
# b = 4 or 9 with probability 1/2, cutoffs of the 9000-row workload, kT 0.005,
# half filling; system i uses seed 3000 + i.
BATCH_SEED0, BATCH_SYSTEMS = 3000, 48


def batched_system(i: int, n_min: int = 200, n_max: int = 4000) -> System:
    rng = np.random.default_rng(BATCH_SEED0 + i)
    n_atoms = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
    b = 4 if rng.uniform() < 0.5 else 9
    return make_system(n_atoms, b, 4.57, 5.99, seed=BATCH_SEED0 + i, kT=0.005)


def make_config(name: str, **over) -> System:
    kw = dict(CONFIGS[name])
    kw.update(over)
    return make_system(**kw)


def spd_on_pattern(pat: BlockPattern, seed: int, lo: float, hi: float) -> np.ndarray:
    """Random symmetric matrix on `pat` with spectrum mapped onto [lo, hi]."""
    rng = np.random.default_rng(seed)
    b = pat.b
    rows = pat.rows()
    cols = pat.col_idx.astype(np.int64)
    upper = rows < cols
    blk = rng.standard_normal((int(upper.sum()), b, b)) * 0.1
    val = np.zeros((pat.nnzb, b, b))
    val[np.nonzero(upper)[0]] = blk
    val[positions_in_pattern(pat, cols[upper], rows[upper])] = np.transpose(blk, (0, 2, 1))
    dpos = positions_in_pattern(pat, np.arange(pat.nb), np.arange(pat.nb))
    d = rng.standard_normal((pat.nb, b, b)) * 0.1
    val[dpos] = d + np.transpose(d, (0, 2, 1))
    w0, w1 = extreme_eigenvalues(pat, val)
    a = (hi - lo) / (w1 - w0)
    val *= a
    val[dpos] += (lo - a * w0) * np.eye(b)[None]
    return val
