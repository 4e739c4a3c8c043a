// HIP kernels (gfx950) for the Chebyshev sparse matrix-function path.
//
// The central kernel is the truncated block product of Sec. "Truncation to a
// fixed sparsity pattern": C = P_C o (A Bt^T), evaluated only on C's block
// pattern.  The Chebyshev recursion of Eq. 4 is run on transposed storage:
// with U_k = T_k^T kept in block CSR (i.e. T_k by block columns, the columns
// that Sec. "Expansion in Chebyshev polynomials" notes are independent),
//     U_{k+1} = P_K o (2 U_k M~) - U_{k-1},
// which is this product with A = U_k, Bt = M~^T, an epilogue
// out = 2 Y - U_{k-1} and, fused into the same pass, the weighted sums of
// Eq. 1 (float64) and the trace Tr T_{k+1} (per-tile float64 partials,
// reduced in fixed order afterwards).
//
// Work decomposition of the product kernel: one workgroup (4 wave64) per tile
// of consecutive block rows of A / C.  The tile's rows of A are copied to LDS
// once (each A block is read from HBM once per product) together with an LDS
// hash table that maps a column index l to the tile's copy of A[i, l] for
// every tile row i.  Each wave then takes output columns j of the tile, walks
// row j of Bt (the row of M~, shared by all tile rows, so every Bt block
// fetched feeds all tile rows that use it) and accumulates
//     Y[i, j] = sum_l A[i, l] Bt[j, l]^T
// with one output element (i, r, s) per lane.  Tiles are mapped to workgroup
// ids so that consecutive tiles (neighbouring atoms) land on the same XCD and
// share their Bt rows in that XCD's L2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "kernels.h"

namespace chess {

namespace {

constexpr int kWG = 256;

__device__ inline unsigned hash_slot(int key, int log2cap) {
    return ((unsigned)key * 2654435761u) >> (32 - log2cap);
}

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block sum over 256 threads (fixed tree).  Every thread of the
// block must call it.  Result valid in thread 0.
__device__ inline double block_sum(double v) {
    __shared__ double red[kWG / 64];
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < kWG / 64; ++w) s += red[w];
    }
    __syncthreads();
    return s;
}

__device__ inline double wave_min(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ inline double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// ---------------------------------------------------------------------------
// masked block product
// ---------------------------------------------------------------------------

// LDS layout of one workgroup (all regions 16-byte aligned):
//   A tile      lds_ablocks * B*B * T   this tile's rows of A
//   hash keys   hcap * int              column l -> index k into the u list
//   hash vals   hcap * short
//   upos        max_u * CMAX * ushort   k -> position of A[i, l] in the tile
//   per wave:   Bt row staging (max_bt_row * B*B * T, only when the row is
//               prefetched through registers) and CMAX hit lists of
//               max_bt_row packed (Bt slot << 16 | A tile position) entries
struct LdsLayout {
    size_t a, hkey, hval, upos, wave, wave_bt, wave_list, total;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

template <typename T, int B, int CMAX, int NW, bool PREF>
__host__ __device__ inline LdsLayout lds_layout(const ProductPlanDev &plan) {
    LdsLayout L;
    const size_t hcap = (size_t)1 << plan.hcap_log2;
    L.a = 0;
    L.hkey = align16((size_t)plan.lds_ablocks * B * B * sizeof(T));
    L.hval = L.hkey + align16(hcap * 4);
    L.upos = L.hval + align16(hcap * 2);
    L.wave = L.upos + align16((size_t)plan.max_u * CMAX * 2);
    L.wave_bt = PREF ? align16((size_t)plan.max_bt_row * B * B * sizeof(T)) : 0;
    L.wave_list = align16((size_t)plan.max_bt_row * CMAX * 4);
    L.total = L.wave + (size_t)NW * (L.wave_bt + L.wave_list);
    return L;
}

__device__ inline void wave_lds_sync() {
    // orders this wave's LDS writes before its later LDS reads (and the reverse)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NT>
__device__ inline double block_sum_n(double v) {
    __shared__ double red[NT / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}

// Copies this tile's rows of A to LDS and builds the LDS hash of its columns.
template <typename T, int B, int CMAX, int NT>
__device__ inline void stage_tile(const ProductPlanDev &plan, const ProductOperands &ops,
                                  unsigned char *smem, const LdsLayout &L, int tile, int row0,
                                  int c) {
    constexpr int BB = B * B;
    const int64_t ab0 = ops.a_rp[row0];
    const int nab = (int)(ops.a_rp[row0 + c] - ab0);
    const int hcap = 1 << plan.hcap_log2;
    T *As = reinterpret_cast<T *>(smem + L.a);
    int *hkey = reinterpret_cast<int *>(smem + L.hkey);
    short *hval = reinterpret_cast<short *>(smem + L.hval);
    unsigned short *upos = reinterpret_cast<unsigned short *>(smem + L.upos);
    const T *Ag = reinterpret_cast<const T *>(ops.a_val) + ab0 * BB;
    if ((BB * sizeof(T)) % 16 == 0) {
        // b = 4: blocks are whole 16-byte chunks and start 16-byte aligned
        const uint4 *src = reinterpret_cast<const uint4 *>(Ag);
        uint4 *dst = reinterpret_cast<uint4 *>(As);
        const int n16 = (int)((size_t)nab * BB * sizeof(T) / 16);
        for (int x = threadIdx.x; x < n16; x += NT) dst[x] = src[x];
    } else {
        const int n = nab * BB;
        for (int x = threadIdx.x; x < n; x += NT) As[x] = Ag[x];
    }
    for (int x = threadIdx.x; x < hcap; x += NT) hkey[x] = -1;
    __syncthreads();
    const int64_t u0 = plan.u_off[tile];
    const int nu = (int)(plan.u_off[tile + 1] - u0);
    const unsigned hmask = (unsigned)hcap - 1u;
    for (int k = threadIdx.x; k < nu; k += NT) {
        const int col = plan.u_cols[u0 + k];
        unsigned h = hash_slot(col, plan.hcap_log2);
        while (true) {
            const int prev = atomicCAS(&hkey[h], -1, col);
            if (prev == -1) {
                hval[h] = (short)k;
                break;
            }
            h = (h + 1u) & hmask;
        }
#pragma unroll
        for (int i = 0; i < CMAX; ++i) upos[k * CMAX + i] = plan.u_pos[(u0 + k) * CMAX + i];
    }
    __syncthreads();
}

// Epilogue for one output element (see Epilogue in kernels.h); the operands
// read from memory were loaded ahead (prevv, accv); wq are the tile's weights
// of the float64 sums.
template <typename T>
__device__ inline void store_output(const ProductOperands &ops, const Epilogue &ep, int64_t off,
                                    T y, T prevv, const double (&accv)[4], const double (&wq)[4],
                                    bool diag, double &tr) {
    T o = (T)ep.alpha * y;
    if (ep.prev) o = fma((T)ep.beta, prevv, o);
    reinterpret_cast<T *>(ops.c_out)[off] = o;
    const double od = (double)o;
#pragma unroll
    for (int qa = 0; qa < 4; ++qa)
        if (qa < ep.nacc) ep.acc[qa][off] = accv[qa] + wq[qa] * od;
    if (ep.hist) reinterpret_cast<T *>(ep.hist)[off] = o;
    if (diag) tr += od;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// The product kernel.  One workgroup per tile of <= CMAX consecutive output
// rows, NW waves; each wave takes output columns j of the tile in turn.  Per
// column: look up every l of row j of Bt in the tile's hash (one lane per l),
// compact the hits of each tile row into an LDS list (ballot + popcount),
// then accumulate Y[i, j] = sum over hits A[i, l] Bt[j, l]^T:
//   MFMA (float, b = 4, CMAX = 4): v_mfma_f32_4x4x1f32 runs 16 independent
//     4x4 outer products; slot g16 = lane / 4 = 4 i + grp takes tile row i and
//     every 4th hit (offset grp) of its list; lane (g16, q) feeds row q of
//     A[i, l] (A operand) and row q of Bt[j, l] (B operand); four MFMAs
//     (k = t = 0..3) form the block product; the four groups of a row are
//     summed across lanes at the end.  Output register v is row v, lane q is
//     column q of the slot's block.
//   VALU (all other types and b): one output element (i, r, s) per lane
//     (several for b = 9), dot products of row r of A[i, l] and row s of Bt[j, l].
// Latency hiding: the (j, Bt row start, length) record of column jj + 2 NW and
// the column indices (and, with PREF, the values) of row j of column jj + NW
// are in flight while column jj is computed; the epilogue operands of column
// jj are loaded before its hits are built.
template <typename T, int B, int CMAX, int NW, bool MFMA, bool PREF>
__global__ __launch_bounds__(64 * NW) void k_product(ProductPlanDev plan, ProductOperands ops,
                                                     Epilogue ep) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    constexpr int BB = B * B;
    constexpr int NT = 64 * NW;
    constexpr int NE = MFMA ? 1 : (CMAX * BB + 63) / 64;
    constexpr int V16 = (BB * (int)sizeof(T)) / 16;          // 16-byte chunks per block (b = 4)
    constexpr int RBV = PREF ? (128 * V16 + 63) / 64 : 1;    // chunks per lane, rows <= 128 blocks
    static_assert(!MFMA || (B == 4 && CMAX == 4 && sizeof(T) == 4), "MFMA path: float, b = 4");
    static_assert(!PREF || B == 4, "register prefetch of Bt rows: b = 4");

    const int ntiles = plan.ntiles;
    const int nt8 = (ntiles + 7) & ~7;
    const int w = blockIdx.x;
    // XCD-aware mapping: workgroup w runs on XCD w % 8; give each XCD a
    // contiguous range of tiles so neighbouring tiles share that XCD's L2.
    const int tile = (w & 7) * (nt8 >> 3) + (w >> 3);
    if (tile >= ntiles) return;
    const LdsLayout L = lds_layout<T, B, CMAX, NW, PREF>(plan);
    const int row0 = plan.tile_row0[tile];
    if (tile_finished(ep, tile, row0)) return;
    const int c = plan.tile_row0[tile + 1] - row0;
    stage_tile<T, B, CMAX, NT>(plan, ops, smem, L, tile, row0, c);
    // weights of the float64 sums: in batches (row_sys set; tiles never
    // straddle systems) those of the tile's system
    double wq[4];
    {
        const int sys = ep.row_sys ? ep.row_sys[row0] : 0;
#pragma unroll
        for (int qa = 0; qa < 4; ++qa)
            wq[qa] = (ep.row_sys && ep.coef_sys[qa]) ? ep.coef_sys[qa][sys] : ep.coef[qa];
    }

    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const T *As = reinterpret_cast<const T *>(smem + L.a);
    unsigned char *wbase = smem + L.wave + (size_t)wave * (L.wave_bt + L.wave_list);
    T *btw = reinterpret_cast<T *>(wbase);
    uint32_t *lists = reinterpret_cast<uint32_t *>(wbase + L.wave_bt);
    const int *hkey = reinterpret_cast<const int *>(smem + L.hkey);
    const short *hval = reinterpret_cast<const short *>(smem + L.hval);
    const unsigned short *upos = reinterpret_cast<const unsigned short *>(smem + L.upos);
    const unsigned hmask = (1u << plan.hcap_log2) - 1u;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int LS = plan.max_bt_row;

    // output elements of this lane: (tile row, row in block, column in block)
    int ei[NE], er[NE], es[NE];
    int64_t cbase[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        if (MFMA) {
            ei[q] = lane >> 4;        // slot / 4
            er[q] = (lane >> 2) & 3;  // hit group = output row written
            es[q] = lane & 3;
        } else {
            const int e = lane + 64 * q;
            ei[q] = e / BB;
            er[q] = (e % BB) / B;
            es[q] = e % B;
        }
        cbase[q] = (ei[q] < c) ? ops.c_rp[row0 + ei[q]] : 0;
    }

    const int64_t j0 = plan.j_off[tile];
    const int nj = (int)(plan.j_off[tile + 1] - j0);
    const int4 *recs = reinterpret_cast<const int4 *>(plan.j_rec);
    const T *BtV = reinterpret_cast<const T *>(ops.bt_val);
    const T *Prev = reinterpret_cast<const T *>(ep.prev);
    double tr = 0.0;

    // pipeline registers: record of the current and next column, column
    // indices and (PREF) values of the current column's Bt row
    int4 rec = make_int4(-1, 0, 0, 0), recN = make_int4(-1, 0, 0, 0);
    uint2 pos = make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu), posN = pos;
    int ci0 = -1, ci1 = -1;
    uint4 bt[RBV];
#define CHESS_LOAD_REC(JJ, R, P)                                                              \
    do {                                                                                       \
        if ((JJ) < nj) {                                                                       \
            R = recs[j0 + (JJ)];                                                               \
            const unsigned short *jp_ = plan.j_pos + (j0 + (JJ)) * CMAX;                       \
            uint32_t v0_ = jp_[0], v1_ = CMAX > 1 ? jp_[1 % CMAX] : 0xFFFFu;                   \
            uint32_t v2_ = CMAX > 2 ? jp_[2 % CMAX] : 0xFFFFu, v3_ = CMAX > 3 ? jp_[3 % CMAX] : 0xFFFFu; \
            P = make_uint2(v0_ | (v1_ << 16), v2_ | (v3_ << 16));                              \
        } else {                                                                               \
            R = make_int4(-1, 0, 0, 0);                                                        \
        }                                                                                      \
    } while (0)
#define CHESS_LOAD_ROW(R, C0, C1, BT)                                                          \
    do {                                                                                       \
        if ((R).x >= 0) {                                                                      \
            C0 = (lane < (R).z) ? ops.bt_ci[(int64_t)(R).y + lane] : -1;                       \
            C1 = (64 + lane < (R).z) ? ops.bt_ci[(int64_t)(R).y + 64 + lane] : -1;             \
            if (PREF) {                                                                        \
                const uint4 *src_ = reinterpret_cast<const uint4 *>(BtV + (int64_t)(R).y * BB); \
                const int n16_ = (R).z * V16;                                                  \
                _Pragma("unroll") for (int v_ = 0; v_ < RBV; ++v_) {                           \
                    const int x_ = v_ * 64 + lane;                                             \
                    BT[v_] = (x_ < n16_) ? src_[x_] : make_uint4(0, 0, 0, 0);                  \
                }                                                                              \
            }                                                                                  \
        }                                                                                      \
    } while (0)
    auto pos_of = [](const uint2 &p, int i) -> unsigned {
        const uint32_t word = (i < 2) ? p.x : p.y;
        return (word >> ((i & 1) * 16)) & 0xFFFFu;
    };

    int jj = wave;
    CHESS_LOAD_REC(jj, rec, pos);
    CHESS_LOAD_ROW(rec, ci0, ci1, bt);
    CHESS_LOAD_REC(jj + NW, recN, posN);
    for (; jj < nj; jj += NW) {
        const int j = rec.x;
        // stage B for the next column, stage A for the one after
        int ciN0 = -1, ciN1 = -1;
        uint4 btN[RBV];
        CHESS_LOAD_ROW(recN, ciN0, ciN1, btN);
        int4 recNN;
        uint2 posNN = make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu);
        CHESS_LOAD_REC(jj + 2 * NW, recNN, posNN);

        // epilogue operands of this column
        int64_t off[NE];
        bool valid[NE];
        T prevv[NE];
        double accv[NE][4];
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const unsigned op = (ei[q] < c) ? pos_of(pos, ei[q]) : 0xFFFFu;
            valid[q] = op != 0xFFFFu;
            off[q] = valid[q] ? (cbase[q] + op) * BB + er[q] * B + es[q] : 0;
            prevv[q] = (valid[q] && Prev) ? Prev[off[q]] : (T)0;
#pragma unroll
            for (int qa = 0; qa < 4; ++qa)
                accv[q][qa] = (valid[q] && qa < ep.nacc) ? ep.acc[qa][off[q]] : 0.0;
        }

        // this column's Bt row to LDS (prefetched through registers)
        if (PREF) {
            uint4 *d16 = reinterpret_cast<uint4 *>(btw);
            const int n16 = rec.z * V16;
#pragma unroll
            for (int v = 0; v < RBV; ++v) {
                const int x = v * 64 + lane;
                if (x < n16) d16[x] = bt[v];
            }
        }
        // hits of every tile row
        int cnt[CMAX];
#pragma unroll
        for (int i = 0; i < CMAX; ++i) cnt[i] = 0;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            if (kk * 64 >= rec.z) break;
            const int l = kk == 0 ? ci0 : ci1;
            int k = -1;
            if (l >= 0) {
                unsigned h = hash_slot(l, plan.hcap_log2);
                while (true) {
                    const int key = hkey[h];
                    if (key == l) {
                        k = hval[h];
                        break;
                    }
                    if (key < 0) break;
                    h = (h + 1u) & hmask;
                }
            }
            const int s = kk * 64 + lane;
#pragma unroll
            for (int i = 0; i < CMAX; ++i) {
                if (pos_of(pos, i) == 0xFFFFu) continue;  // no output block (i, j)
                const unsigned short pa = (k >= 0) ? upos[k * CMAX + i] : (unsigned short)0xFFFF;
                const bool hit = pa != 0xFFFF;
                const uint64_t m = __ballot(hit);
                if (hit) lists[i * LS + cnt[i] + __popcll(m & lt_mask)] = ((uint32_t)s << 16) | pa;
                cnt[i] += __popcll(m);
            }
        }
        // rows longer than 128 blocks: remaining slots one round at a time
        for (int base = 128; base < rec.z; base += 64) {
            const int s = base + lane;
            int k = -1;
            if (s < rec.z) {
                const int l = ops.bt_ci[(int64_t)rec.y + s];
                unsigned h = hash_slot(l, plan.hcap_log2);
                while (true) {
                    const int key = hkey[h];
                    if (key == l) {
                        k = hval[h];
                        break;
                    }
                    if (key < 0) break;
                    h = (h + 1u) & hmask;
                }
            }
#pragma unroll
            for (int i = 0; i < CMAX; ++i) {
                if (pos_of(pos, i) == 0xFFFFu) continue;
                const unsigned short pa = (k >= 0) ? upos[k * CMAX + i] : (unsigned short)0xFFFF;
                const bool hit = pa != 0xFFFF;
                const uint64_t m = __ballot(hit);
                if (hit) lists[i * LS + cnt[i] + __popcll(m & lt_mask)] = ((uint32_t)s << 16) | pa;
                cnt[i] += __popcll(m);
            }
        }
        wave_lds_sync();

        T y[NE];
        if (MFMA) {
            const int mi = lane >> 4, grp = (lane >> 2) & 3, q = lane & 3;
            int nmax = 0, nmine = 0;
#pragma unroll
            for (int i = 0; i < CMAX; ++i) {
                nmax = max(nmax, cnt[i]);
                if (i == mi) nmine = cnt[i];
            }
            const uint32_t *mylist = lists + mi * LS;
            const float *bsrc = PREF ? reinterpret_cast<const float *>(btw)
                                     : reinterpret_cast<const float *>(BtV) + (int64_t)rec.y * BB;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            const int iters = (nmax + 3) >> 2;
            for (int it = 0; it < iters; ++it) {
                const int h = grp + 4 * it;
                f32x4 a = {0.f, 0.f, 0.f, 0.f}, bb = {0.f, 0.f, 0.f, 0.f};
                if (h < nmine) {
                    const uint32_t e = mylist[h];
                    a = *reinterpret_cast<const f32x4 *>(reinterpret_cast<const float *>(As) + (int)(e & 0xFFFF) * BB + q * B);
                    bb = *reinterpret_cast<const f32x4 *>(bsrc + (int)(e >> 16) * BB + q * B);
                }
                acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a[0], bb[0], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a[1], bb[1], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a[2], bb[2], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a[3], bb[3], acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                acc[v] += __shfl_xor(acc[v], 4, 64);
                acc[v] += __shfl_xor(acc[v], 8, 64);
            }
            float yy = acc[0];
            if (grp == 1) yy = acc[1];
            if (grp == 2) yy = acc[2];
            if (grp == 3) yy = acc[3];
            y[0] = (T)yy;
        } else {
            int n[NE];
            const uint32_t *li[NE];
            int nmax = 0;
#pragma unroll
            for (int q = 0; q < NE; ++q) {
                int nq = 0;
#pragma unroll
                for (int i = 0; i < CMAX; ++i)
                    if (i == ei[q]) nq = cnt[i];
                n[q] = valid[q] ? nq : 0;
                li[q] = lists + (ei[q] < CMAX ? ei[q] : 0) * LS;
                nmax = max(nmax, n[q]);
                y[q] = (T)0;
            }
            const T *bsrc = PREF ? btw : BtV + (int64_t)rec.y * BB;
            for (int h = 0; h < nmax; ++h) {
#pragma unroll
                for (int q = 0; q < NE; ++q) {
                    if (h < n[q]) {
                        const uint32_t e = li[q][h];
                        const T *a = As + (int)(e & 0xFFFF) * BB + er[q] * B;
                        const T *bs = bsrc + (int64_t)(e >> 16) * BB + es[q] * B;
                        T s = (T)0;
#pragma unroll
                        for (int t = 0; t < B; ++t) s = fma(a[t], bs[t], s);
                        y[q] += s;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NE; ++q)
            if (valid[q])
                store_output<T>(ops, ep, off[q], y[q], prevv[q], accv[q], wq,
                                row0 + ei[q] == j && er[q] == es[q], tr);
        // the next column overwrites this wave's staging and lists
        wave_lds_sync();
        rec = recN;
        pos = posN;
        ci0 = ciN0;
        ci1 = ciN1;
#pragma unroll
        for (int v = 0; v < RBV; ++v) bt[v] = btN[v];
        recN = recNN;
        posN = posNN;
    }
#undef CHESS_LOAD_REC
#undef CHESS_LOAD_ROW
    if (ep.trace_partial) {
        const double s = block_sum_n<NT>(tr);
        if (threadIdx.x == 0) ep.trace_partial[tile] = s;
    }
}

// Kernel variant for (T, b, CMAX): waves per workgroup, MFMA, register prefetch.
template <typename T, int B, int CMAX>
struct Variant {
    static constexpr bool MFMA = std::is_same<T, float>::value && B == 4 && CMAX == 4;
    static constexpr int NW = sizeof(T) == 4 ? 8 : 4;
};

template <typename T, int B, int CMAX, bool PREF>
size_t product_lds_p(const ProductPlanDev &plan) {
    return lds_layout<T, B, CMAX, Variant<T, B, CMAX>::NW, PREF>(plan).total;
}

template <typename T, int B, int CMAX>
size_t product_lds(const ProductPlanDev &plan) {
    return (B == 4 && plan.stage_bt) ? product_lds_p<T, B, CMAX, true>(plan)
                                     : product_lds_p<T, B, CMAX, false>(plan);
}

template <typename T, int B, int CMAX, bool PREF>
hipError_t launch_product_p(const ProductPlanDev &plan, const ProductOperands &ops,
                            const Epilogue &ep, hipStream_t st) {
    constexpr int NW = Variant<T, B, CMAX>::NW;
    constexpr bool MFMA = Variant<T, B, CMAX>::MFMA;
    const size_t lds = product_lds_p<T, B, CMAX, PREF>(plan);
    const void *fn = (const void *)k_product<T, B, CMAX, NW, MFMA, PREF>;
    // raise the dynamic LDS limit once per kernel instantiation (and device
    // ordinal), only when a launch needs more than the default 64 KB
    static int raised_device = -1;
    static size_t raised_to = 0;
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (lds > 65536 && (raised_device != dev || raised_to < lds)) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        raised_device = dev;
        raised_to = lds;
    }
    const int nt8 = (plan.ntiles + 7) & ~7;
    hipLaunchKernelGGL((k_product<T, B, CMAX, NW, MFMA, PREF>), dim3(nt8), dim3(64 * NW), lds, st,
                       plan, ops, ep);
    return hipGetLastError();
}

template <typename T, int B, int CMAX>
hipError_t launch_product_t(const ProductPlanDev &plan, const ProductOperands &ops,
                            const Epilogue &ep, hipStream_t st) {
    if (plan.ntiles == 0) return hipSuccess;
    if constexpr (B == 4) {
        if (plan.stage_bt) return launch_product_p<T, B, CMAX, true>(plan, ops, ep, st);
    }
    return launch_product_p<T, B, CMAX, false>(plan, ops, ep, st);
}

template <typename T, int B>
hipError_t dispatch_cmax(const ProductPlanDev &plan, const ProductOperands &ops,
                         const Epilogue &ep, hipStream_t st, size_t *lds_out) {
    switch (plan.cmax) {
        case 1:
            if (lds_out) { *lds_out = product_lds<T, B, 1>(plan); return hipSuccess; }
            return launch_product_t<T, B, 1>(plan, ops, ep, st);
        case 2:
            if (lds_out) { *lds_out = product_lds<T, B, 2>(plan); return hipSuccess; }
            return launch_product_t<T, B, 2>(plan, ops, ep, st);
        case 4:
            if (lds_out) { *lds_out = product_lds<T, B, 4>(plan); return hipSuccess; }
            return launch_product_t<T, B, 4>(plan, ops, ep, st);
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t dispatch_product(int dtype, int b, const ProductPlanDev &plan,
                            const ProductOperands &ops, const Epilogue &ep, hipStream_t st,
                            size_t *lds_out) {
    if (dtype == 0 && b == 4) return dispatch_cmax<double, 4>(plan, ops, ep, st, lds_out);
    if (dtype == 0 && b == 9) return dispatch_cmax<double, 9>(plan, ops, ep, st, lds_out);
    if (dtype == 1 && b == 4) return dispatch_cmax<float, 4>(plan, ops, ep, st, lds_out);
    if (dtype == 1 && b == 9) return dispatch_cmax<float, 9>(plan, ops, ep, st, lds_out);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_fill_identity(int b, int64_t nnzb, const int32_t *brow, const int32_t *bcol,
                                T *out) {
    const int64_t bb = (int64_t)b * b;
    const int64_t n = nnzb * bb;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = x / bb;
        const int e = (int)(x % bb);
        const int r = e / b, s = e % b;
        out[x] = (brow[p] == bcol[p] && r == s) ? (T)1 : (T)0;
    }
}

template <typename T>
__global__ void k_scatter_blocks(int b, int64_t nnzb_in, const int64_t *map, const double *in,
                                 T *out, int transpose) {
    const int64_t bb = (int64_t)b * b;
    const int64_t n = nnzb_in * bb;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = x / bb;
        const int e = (int)(x % bb);
        const int r = e / b, s = e % b;
        const int64_t dst = map[p] * bb + (transpose ? (s * b + r) : e);
        out[dst] = (T)in[x];
    }
}

__global__ void k_scale_shift(int b, int64_t nnzb, const int32_t *brow, const int32_t *bcol,
                              const double *in, double *out, double sigma, double tau) {
    const int64_t bb = (int64_t)b * b;
    const int64_t n = nnzb * bb;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = x / bb;
        const int e = (int)(x % bb);
        const int r = e / b, s = e % b;
        const double d = (brow[p] == bcol[p] && r == s) ? tau : 0.0;
        out[x] = sigma * (in[x] - d);
    }
}

// Block-diagonal batches: per block row I the system row_sys[I] gives its own
// sigma and tau.
__global__ void k_scale_shift_rows(int b, int64_t nnzb, const int32_t *brow, const int32_t *bcol,
                                   const int32_t *row_sys, const double *sigma, const double *tau,
                                   const double *in, double *out) {
    const int64_t bb = (int64_t)b * b;
    const int64_t n = nnzb * bb;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = x / bb;
        const int e = (int)(x % bb);
        const int r = e / b, s = e % b;
        const int sys = row_sys[brow[p]];
        const double d = (brow[p] == bcol[p] && r == s) ? tau[sys] : 0.0;
        out[x] = sigma[sys] * (in[x] - d);
    }
}

// out[k * nseg + s] = sum of part[k * ntiles + t] over t in [seg[s], seg[s+1]),
// in order; grid (nseg, nk).
__global__ void k_segment_sum(int ntiles, int nseg, const int32_t *seg, const double *part,
                              double *out) {
    const int sg = blockIdx.x, k = blockIdx.y;
    const double *p = part + (int64_t)k * ntiles;
    double s = 0.0;
    for (int t = seg[sg] + threadIdx.x; t < seg[sg + 1]; t += blockDim.x) s += p[t];
    s = block_sum(s);
    if (threadIdx.x == 0) out[(int64_t)k * nseg + sg] = s;
}

__global__ void k_symmetrize(int b, int64_t nnzb, const int64_t *tmap, const double *in,
                             double *out) {
    const int64_t bb = (int64_t)b * b;
    const int64_t n = nnzb * bb;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = x / bb;
        const int e = (int)(x % bb);
        const int r = e / b, s = e % b;
        out[x] = 0.5 * (in[x] + in[tmap[p] * bb + s * b + r]);
    }
}

template <typename T>
__global__ void k_axpby_to_f64(int64_t n, double a0, const T *t0, double a1, const T *t1,
                               double *acc) {
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        double v = a0 * (double)t0[x];
        if (t1) v += a1 * (double)t1[x];
        acc[x] = v;
    }
}

template <typename T>
__global__ void k_recombine(int64_t n, int nk, const T *hist, const double *coef, double *acc) {
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        const T *h = hist + x;
        for (int k = 0; k < nk; ++k) s += coef[k] * (double)h[(int64_t)k * n];
        acc[x] = s;
    }
}

template <typename T>
__global__ void k_trace(int b, int nb, const int64_t *diag_idx, const T *val, double *part) {
    double s = 0.0;
    const int64_t bb = (int64_t)b * b;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x) {
        const T *d = val + diag_idx[i] * bb;
        for (int r = 0; r < b; ++r) s += (double)d[r * b + r];
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Per-workgroup partials of sum x^2 (part[w]) and sum x y (part[nparts + w])
// over n values, accumulated in float64; 16-byte loads (n is a multiple of
// 16 / sizeof(T): whole 4 x 4 or 9 x 9 block arrays of at least 16 values
// are not, so a scalar tail takes the rest).
template <typename T>
__global__ void k_dot_pair(int64_t n, const T *x, const T *y, double *part) {
    typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type V;
    constexpr int W = 16 / sizeof(T);
    const int nparts = gridDim.x;
    const int64_t nv = n / W;
    const V *xv = reinterpret_cast<const V *>(x);
    const V *yv = reinterpret_cast<const V *>(y);
    double sq = 0.0, xy = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nv; i += stride) {
        const V a = xv[i], c = yv[i];
        if constexpr (W == 4) {
            sq += (double)a.x * a.x + (double)a.y * a.y + (double)a.z * a.z + (double)a.w * a.w;
            xy += (double)a.x * c.x + (double)a.y * c.y + (double)a.z * c.z + (double)a.w * c.w;
        } else {
            sq += a.x * a.x + a.y * a.y;
            xy += a.x * c.x + a.y * c.y;
        }
    }
    for (int64_t i = nv * W + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
        sq += (double)x[i] * x[i];
        xy += (double)x[i] * y[i];
    }
    sq = block_sum(sq);
    xy = block_sum(xy);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = sq;
        part[nparts + blockIdx.x] = xy;
    }
}

__global__ void k_reduce_rows(int nparts, const double *part, double *out) {
    double s = 0.0;
    const double *p = part + (int64_t)blockIdx.x * nparts;
    for (int t = threadIdx.x; t < nparts; t += blockDim.x) s += p[t];
    s = block_sum(s);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ void k_gershgorin(int b, int nb, const int64_t *rp, const int32_t *ci,
                             const double *val, double *part_lo, double *part_hi) {
    double lo = 1e300, hi = -1e300;
    const int n = nb * b;
    const int bb = b * b;
    for (int R = blockIdx.x * blockDim.x + threadIdx.x; R < n; R += gridDim.x * blockDim.x) {
        const int I = R / b, r = R % b;
        double rad = 0.0, d = 0.0;
        for (int64_t p = rp[I]; p < rp[I + 1]; ++p) {
            const double *blk = val + p * bb + r * b;
            for (int s = 0; s < b; ++s) {
                if (ci[p] == I && s == r)
                    d = blk[s];
                else
                    rad += fabs(blk[s]);
            }
        }
        lo = fmin(lo, d - rad);
        hi = fmax(hi, d + rad);
    }
    __shared__ double slo[kWG / 64], shi[kWG / 64];
    lo = wave_min(lo);
    hi = wave_max(hi);
    if ((threadIdx.x & 63) == 0) {
        slo[threadIdx.x >> 6] = lo;
        shi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWG / 64; ++w) {
            lo = fmin(lo, slo[w]);
            hi = fmax(hi, shi[w]);
        }
        lo = fmin(slo[0], lo);
        hi = fmax(shi[0], hi);
        part_lo[blockIdx.x] = lo;
        part_hi[blockIdx.x] = hi;
    }
}

__global__ void k_minmax(int nparts, const double *plo, const double *phi, double *out2) {
    double lo = 1e300, hi = -1e300;
    for (int t = threadIdx.x; t < nparts; t += blockDim.x) {
        lo = fmin(lo, plo[t]);
        hi = fmax(hi, phi[t]);
    }
    __shared__ double slo[kWG / 64], shi[kWG / 64];
    lo = wave_min(lo);
    hi = wave_max(hi);
    if ((threadIdx.x & 63) == 0) {
        slo[threadIdx.x >> 6] = lo;
        shi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 0; w < kWG / 64; ++w) {
            lo = fmin(lo, slo[w]);
            hi = fmax(hi, shi[w]);
        }
        out2[0] = lo;
        out2[1] = hi;
    }
}

__global__ void k_spmv(int b, int nb, const int64_t *rp, const int32_t *ci, const double *val,
                       const double *x, double *y) {
    const int n = nb * b;
    const int bb = b * b;
    for (int R = blockIdx.x * blockDim.x + threadIdx.x; R < n; R += gridDim.x * blockDim.x) {
        const int I = R / b, r = R % b;
        double s = 0.0;
        for (int64_t p = rp[I]; p < rp[I + 1]; ++p) {
            const double *blk = val + p * bb + r * b;
            const double *xs = x + (int64_t)ci[p] * b;
            for (int t = 0; t < b; ++t) s += blk[t] * xs[t];
        }
        y[R] = s;
    }
}

__global__ void k_multidot(int64_t n, const double *V, const double *w, double *part,
                           int nparts) {
    const int j = blockIdx.y;
    const double *v = V + (int64_t)j * n;
    double s = 0.0;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        s += v[x] * w[x];
    s = block_sum(s);
    if (threadIdx.x == 0) part[(int64_t)j * nparts + blockIdx.x] = s;
}

__global__ void k_multiaxpy(int m, int64_t n, const double *V, const double *h, double *w) {
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        double s = w[x];
        for (int j = 0; j < m; ++j) s -= h[j] * V[(int64_t)j * n + x];
        w[x] = s;
    }
}

__global__ void k_normalize(int64_t n, const double *x, const double *nrm2, double *y) {
    const double inv = 1.0 / sqrt(*nrm2);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = x[i] * inv;
}

__global__ void k_trace_product(int b, int64_t nnzb_s, const int64_t *kmap_t, const double *K,
                                const double *S, double *part) {
    const int64_t bb = (int64_t)b * b;
    const int64_t n = nnzb_s * bb;
    double acc = 0.0;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = x / bb;
        const int e = (int)(x % bb);
        const int r = e / b, s = e % b;
        // S[q] is block (J, I); K block (I, J) element (s, r) pairs with S (r, s)
        acc += S[x] * K[kmap_t[q] * bb + s * b + r];
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ void k_zero_words(int64_t n, uint32_t *p) {
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        p[x] = 0u;
}

template <typename T>
__global__ void k_convert(int64_t n, const double *in, T *out) {
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        out[x] = (T)in[x];
}

inline int grid_for(int64_t n) {
    int64_t g = (n + kWG - 1) / kWG;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

hipError_t launch_masked_product(int dtype, int b, const ProductPlanDev &plan,
                                 const ProductOperands &ops, const Epilogue &ep,
                                 hipStream_t st) {
    return dispatch_product(dtype, b, plan, ops, ep, st, nullptr);
}

size_t masked_product_lds_bytes(int dtype, int b, const ProductPlanDev &plan) {
    size_t lds = 0;
    if (dispatch_product(dtype, b, plan, ProductOperands{}, Epilogue{}, nullptr, &lds) !=
        hipSuccess)
        return (size_t)-1;
    return lds;
}

hipError_t launch_fill_identity(int dtype, int b, int64_t nnzb, const int32_t *brow,
                                const int32_t *bcol, void *out, hipStream_t st) {
    const int g = grid_for(nnzb * b * b);
    if (dtype == 0)
        hipLaunchKernelGGL(k_fill_identity<double>, dim3(g), dim3(kWG), 0, st, b, nnzb, brow,
                           bcol, (double *)out);
    else
        hipLaunchKernelGGL(k_fill_identity<float>, dim3(g), dim3(kWG), 0, st, b, nnzb, brow, bcol,
                           (float *)out);
    return hipGetLastError();
}

hipError_t launch_scatter_blocks(int dtype_out, int b, int64_t nnzb_in, const int64_t *map,
                                 const double *in, void *out, int transpose, hipStream_t st) {
    const int g = grid_for(nnzb_in * b * b);
    if (dtype_out == 0)
        hipLaunchKernelGGL(k_scatter_blocks<double>, dim3(g), dim3(kWG), 0, st, b, nnzb_in, map,
                           in, (double *)out, transpose);
    else
        hipLaunchKernelGGL(k_scatter_blocks<float>, dim3(g), dim3(kWG), 0, st, b, nnzb_in, map,
                           in, (float *)out, transpose);
    return hipGetLastError();
}

hipError_t launch_scale_shift_rows(int b, int64_t nnzb, const int32_t *brow, const int32_t *bcol,
                                  const int32_t *row_sys, const double *sigma, const double *tau,
                                  const double *in, double *out, hipStream_t st) {
    if (nnzb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_shift_rows, dim3(grid_for(nnzb * b * b)), dim3(kWG), 0, st, b, nnzb,
                       brow, bcol, row_sys, sigma, tau, in, out);
    return hipGetLastError();
}

hipError_t launch_segment_sum(int nk, int ntiles, int nseg, const int32_t *seg, const double *part,
                              double *out, hipStream_t st) {
    if (nk <= 0 || nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_segment_sum, dim3(nseg, nk), dim3(kWG), 0, st, ntiles, nseg, seg, part, out);
    return hipGetLastError();
}

hipError_t launch_scale_shift(int b, int64_t nnzb, const int32_t *brow, const int32_t *bcol,
                              const double *in, double *out, double sigma, double tau,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_scale_shift, dim3(grid_for(nnzb * b * b)), dim3(kWG), 0, st, b, nnzb,
                       brow, bcol, in, out, sigma, tau);
    return hipGetLastError();
}

hipError_t launch_symmetrize(int b, int64_t nnzb, const int64_t *tmap, const double *in,
                             double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_symmetrize, dim3(grid_for(nnzb * b * b)), dim3(kWG), 0, st, b, nnzb,
                       tmap, in, out);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t st) {
    // a fill kernel rather than a memset node, so that the sequence stays
    // valid inside a captured HIP graph
    if (bytes == 0) return hipSuccess;
    if (bytes % 4 != 0) return hipErrorInvalidValue;
    const int64_t n = (int64_t)(bytes / 4);
    hipLaunchKernelGGL(k_zero_words, dim3(grid_for(n)), dim3(kWG), 0, st, n, (uint32_t *)p);
    return hipGetLastError();
}

hipError_t launch_axpby_to_f64(int dtype, int64_t n, double a0, const void *t0, double a1,
                               const void *t1, double *acc, hipStream_t st) {
    const int g = grid_for(n);
    if (dtype == 0)
        hipLaunchKernelGGL(k_axpby_to_f64<double>, dim3(g), dim3(kWG), 0, st, n, a0,
                           (const double *)t0, a1, (const double *)t1, acc);
    else
        hipLaunchKernelGGL(k_axpby_to_f64<float>, dim3(g), dim3(kWG), 0, st, n, a0,
                           (const float *)t0, a1, (const float *)t1, acc);
    return hipGetLastError();
}

hipError_t launch_recombine(int dtype, int64_t n, int nk, const void *hist, const double *coef,
                            double *acc, hipStream_t st) {
    const int g = grid_for(n);
    if (dtype == 0)
        hipLaunchKernelGGL(k_recombine<double>, dim3(g), dim3(kWG), 0, st, n, nk,
                           (const double *)hist, coef, acc);
    else
        hipLaunchKernelGGL(k_recombine<float>, dim3(g), dim3(kWG), 0, st, n, nk,
                           (const float *)hist, coef, acc);
    return hipGetLastError();
}

hipError_t launch_trace(int dtype, int b, int nb, const int64_t *diag_idx, const void *val,
                        double *out_partial, int nparts, hipStream_t st) {
    if (dtype == 0)
        hipLaunchKernelGGL(k_trace<double>, dim3(nparts), dim3(kWG), 0, st, b, nb, diag_idx,
                           (const double *)val, out_partial);
    else
        hipLaunchKernelGGL(k_trace<float>, dim3(nparts), dim3(kWG), 0, st, b, nb, diag_idx,
                           (const float *)val, out_partial);
    return hipGetLastError();
}

hipError_t launch_dot_pair(int dtype, int64_t n, const void *x, const void *y, double *part,
                           int nparts, hipStream_t st) {
    if (dtype == 0)
        hipLaunchKernelGGL(k_dot_pair<double>, dim3(nparts), dim3(kWG), 0, st, n, (const double *)x,
                           (const double *)y, part);
    else
        hipLaunchKernelGGL(k_dot_pair<float>, dim3(nparts), dim3(kWG), 0, st, n, (const float *)x,
                           (const float *)y, part);
    return hipGetLastError();
}

hipError_t launch_reduce_rows(int nrows, int nparts, const double *part, double *out,
                              hipStream_t st) {
    if (nrows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_rows, dim3(nrows), dim3(kWG), 0, st, nparts, part, out);
    return hipGetLastError();
}

hipError_t launch_gershgorin(int b, int nb, const int64_t *rp, const int32_t *ci,
                             const double *val, double *part_lo, double *part_hi, int nparts,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_gershgorin, dim3(nparts), dim3(kWG), 0, st, b, nb, rp, ci, val,
                       part_lo, part_hi);
    return hipGetLastError();
}

hipError_t launch_minmax(int nparts, const double *part_lo, const double *part_hi, double *out2,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_minmax, dim3(1), dim3(kWG), 0, st, nparts, part_lo, part_hi, out2);
    return hipGetLastError();
}

hipError_t launch_spmv(int b, int nb, const int64_t *rp, const int32_t *ci, const double *val,
                       const double *x, double *y, hipStream_t st) {
    hipLaunchKernelGGL(k_spmv, dim3(grid_for((int64_t)nb * b)), dim3(kWG), 0, st, b, nb, rp, ci,
                       val, x, y);
    return hipGetLastError();
}

hipError_t launch_multidot(int m, int64_t n, const double *V, const double *w, double *part,
                           int nparts, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_multidot, dim3(nparts, m), dim3(kWG), 0, st, n, V, w, part, nparts);
    return hipGetLastError();
}

hipError_t launch_multiaxpy(int m, int64_t n, const double *V, const double *h, double *w,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_multiaxpy, dim3(grid_for(n)), dim3(kWG), 0, st, m, n, V, h, w);
    return hipGetLastError();
}

hipError_t launch_normalize(int64_t n, const double *x, const double *nrm2, double *y,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_normalize, dim3(grid_for(n)), dim3(kWG), 0, st, n, x, nrm2, y);
    return hipGetLastError();
}

hipError_t launch_trace_product(int b, int64_t nnzb_s, const int64_t *kmap_t, const double *K,
                                const double *S, double *part, int nparts, hipStream_t st) {
    hipLaunchKernelGGL(k_trace_product, dim3(nparts), dim3(kWG), 0, st, b, nnzb_s, kmap_t, K, S,
                       part);
    return hipGetLastError();
}

hipError_t launch_convert(int dtype_out, int64_t n, const double *in, void *out,
                          hipStream_t st) {
    const int g = grid_for(n);
    if (dtype_out == 0)
        hipLaunchKernelGGL(k_convert<double>, dim3(g), dim3(kWG), 0, st, n, in, (double *)out);
    else
        hipLaunchKernelGGL(k_convert<float>, dim3(g), dim3(kWG), 0, st, n, in, (float *)out);
    return hipGetLastError();
}

}  // namespace chess
