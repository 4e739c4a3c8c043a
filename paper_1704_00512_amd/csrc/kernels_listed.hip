// The Chebyshev-step product with precomputed hit lists.
//
// A chain runs the same truncated product C = P_C o (A Bt^T) hundreds to
// thousands of times on one fixed pattern triple, so every intersection
// "which l contribute to output block (i, j)" is worked out once, on the host,
// and stored as a compact list per (row tile, output column j, tile row i):
// one entry per contributing l holding the block's position inside row i of A
// and inside row j of Bt (8 + 8 bits, or 16 + 16 bits when a row has more than
// 255 blocks).  Each step then streams these lists instead of searching.
//
// Work decomposition: one workgroup (NW wave64) per tile of <= CMAX
// consecutive rows; the tile's rows of A are copied to LDS once.  Each wave
// takes output columns j of the tile in turn.  For column j it stages row j of
// Bt and the column's hit lists in its LDS area (both prefetched through
// registers one column ahead, the column record two columns ahead), then
//   MFMA (float, b = 4, CMAX = 4): v_mfma_f32_4x4x1f32 performs 16
//     independent 4x4 outer products; slot = lane / 4 = 4 i + grp takes tile
//     row i and every 4th hit (offset grp); lane (slot, q) supplies row q of
//     A[i, l] as the A operand and row q of Bt[j, l] as the B operand; four
//     MFMAs (k = t = 0..3) give the block product A[i, l] Bt[j, l]^T; the four
//     groups of a row are summed across lanes.  Result register v is row v,
//     lane q column q of the slot's block.
//   VALU (float64, or b = 9): one output element (i, r, s) per lane (several
//     for b = 9), dot products of row r of A[i, l] and row s of Bt[j, l].
// The epilogue (kernels.h, Epilogue) is fused: 2 Y - T_{k-1}, the float64
// weighted sums of Eq. 1, a history copy and per-tile trace partials.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "kernels.h"

namespace chess {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

// Streamed data (A tile rows, records, hit lists, T_{k-1}, accumulators,
// outputs) is touched once per launch; with NTH it carries the non-temporal
// hint so that L2 keeps the rows of Bt, which many tiles re-read.
template <bool NTH, typename V>
__device__ inline V ld_stream(const V *p) {
    if constexpr (NTH)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}
template <bool NTH, typename V>
__device__ inline void st_stream(V *p, V v) {
    if constexpr (NTH)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~(size_t)15; }

constexpr int kEntWords = 4;  // prefetched 4-byte words of entries per lane (<= 1 KB per column)

struct ListedLds {
    size_t a, wave, wave_bt, wave_ent, total;
};

template <typename T, int B, int NW, int EW, bool BD>
__host__ __device__ inline ListedLds listed_lds(const ListedPlanDev &p) {
    ListedLds L;
    L.a = 0;
    // A tile, then one block of zeros (the operand of padded MFMA slots)
    L.wave = al16((size_t)(p.lds_ablocks + 1) * B * B * sizeof(T));
    // Bt rows are staged only for b = 4 (16-byte chunks); b = 9 reads them from global memory
    L.wave_bt = (!BD && (B * B * sizeof(T)) % 16 == 0)
                    ? (((size_t)p.max_bt_row * B * B * sizeof(T) / 16 + 63) / 64) * 64 * 16
                    : 0;
    L.wave_ent = al16((size_t)kEntWords * 64 * 4);
    L.total = L.wave + (size_t)NW * (L.wave_bt + L.wave_ent);
    return L;
}

__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double wsum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int NT>
__device__ inline double bsum(double v) {
    __shared__ double red[NT / 64];
    v = wsum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}

// entry decoding: position in A row i and in Bt row j
template <int EW>
__device__ inline void decode(const void *ent, int idx, int &pa, int &sl) {
    if (EW == 1) {
        const uint16_t e = reinterpret_cast<const uint16_t *>(ent)[idx];
        pa = e & 0xFF;
        sl = e >> 8;
    } else {
        const uint32_t e = reinterpret_cast<const uint32_t *>(ent)[idx];
        pa = e & 0xFFFF;
        sl = e >> 16;
    }
}

template <typename T, int B, int CMAX, int NW, int MODE, int EW, bool BD, bool PIPE, bool NTH,
          int G, bool SB, int MAXACC, bool PAD>
__global__ __launch_bounds__(64 * NW) void k_listed(ListedPlanDev plan, ProductOperands ops,
                                                    Epilogue ep) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    constexpr int BB = B * B;
    constexpr int NT = 64 * NW;
    constexpr bool MFMA = MODE == 1;
    constexpr bool MF64 = MODE == 2;
    constexpr int kEntMax = kEntWords * 64 * 4 / (2 * EW);  // entries in a wave's list area
    constexpr int NE = (MFMA || MF64) ? 1 : (CMAX * BB + 63) / 64;
    // BD: MFMA operands of Bt come straight from global memory (L1/L2) and
    // Bt rows are not staged in LDS
    constexpr bool V16OK = !BD && (BB * sizeof(T)) % 16 == 0;
    constexpr int V16 = V16OK ? (BB * (int)sizeof(T)) / 16 : 1;
    constexpr int RBV = V16OK ? (128 * V16 + 63) / 64 : 1;  // Bt rows up to 128 blocks
    static_assert(!MFMA || (B == 4 && CMAX == 4 && sizeof(T) == 4), "MFMA path: float, b = 4");
    static_assert(!MF64 || (B == 4 && CMAX == 4 && sizeof(T) == 8), "MFMA64 path: double, b = 4");
    static_assert(!BD || MFMA || MF64, "direct Bt operands: MFMA paths only");
    static_assert(!PIPE || (MFMA && BD), "pipelined hit groups: float32 MFMA path with direct operands");
    static_assert(G == 4 || (MFMA && BD && !PIPE && SB), "larger hit groups: float32 MFMA path with direct operands");
    static_assert(!PAD || G > 4, "padded hit groups: larger groups only");
    static_assert(!SB || ((MFMA || MF64) && BD), "scheduling barrier: MFMA paths with direct operands");

    const int ntiles = plan.ntiles;
    const int nt8 = (ntiles + 7) & ~7;
    const int w = blockIdx.x;
    // XCD-aware mapping: workgroup w runs on XCD w % 8; each XCD gets a
    // contiguous range of tiles so neighbouring tiles share its L2.
    const int tile = (w & 7) * (nt8 >> 3) + (w >> 3);
    if (tile >= ntiles) return;
    const ListedLds L = listed_lds<T, B, NW, EW, BD>(plan);
    const int row0 = plan.tile_row0[tile];
    if (tile_finished(ep, tile, row0)) return;
    const int c = plan.tile_row0[tile + 1] - row0;
    const int64_t ab0 = ops.a_rp[row0];

    // tile rows of A -> LDS
    T *As = reinterpret_cast<T *>(smem + L.a);
    {
        const int nab = (int)(ops.a_rp[row0 + c] - ab0);
        const T *Ag = reinterpret_cast<const T *>(ops.a_val) + ab0 * BB;
        if ((BB * sizeof(T)) % 16 == 0) {
            const u32x4 *src = reinterpret_cast<const u32x4 *>(Ag);
            u32x4 *dst = reinterpret_cast<u32x4 *>(As);
            const int n16 = nab * (int)((BB * sizeof(T)) / 16);
            for (int x = threadIdx.x; x < n16; x += NT) dst[x] = ld_stream<NTH>(src + x);
        } else {
            for (int x = threadIdx.x; x < nab * BB; x += NT) As[x] = Ag[x];
        }
        for (int x = threadIdx.x; x < BB; x += NT) As[(size_t)plan.lds_ablocks * BB + x] = (T)0;
    }
    int rstart[CMAX];
    int64_t cbase_i[CMAX];
#pragma unroll
    for (int i = 0; i < CMAX; ++i) {
        rstart[i] = (i < c) ? (int)(ops.a_rp[row0 + i] - ab0) : 0;
        cbase_i[i] = (i < c) ? ops.c_rp[row0 + i] : 0;
    }
    __syncthreads();

    // the wave index is uniform: keep it (and everything derived from the
    // column records) in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    unsigned char *wb = smem + L.wave + (size_t)wave * (L.wave_bt + L.wave_ent);
    T *btw = reinterpret_cast<T *>(wb);
    unsigned char *entw = wb + L.wave_bt;

    // this lane's output elements
    int ei[NE], er[NE], es[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        if (MFMA) {
            ei[q] = lane >> 4;
            er[q] = (lane >> 2) & 3;
            es[q] = lane & 3;
        } else if (MF64) {
            // v_mfma_f64_4x4x4f64 result: lane 16 r + 4 blk + s holds D[blk][r][s]
            ei[q] = (lane >> 2) & 3;
            er[q] = lane >> 4;
            es[q] = lane & 3;
        } else {
            const int e = lane + 64 * q;
            ei[q] = e / BB;
            er[q] = (e % BB) / B;
            es[q] = e % B;
        }
    }

    const int64_t j0 = plan.j_off[tile];
    const int nj = (int)(plan.j_off[tile + 1] - j0);
    // accumulator weights of this tile (one system per tile in batches)
    double wq[MAXACC];
    {
        const int sys = ep.row_sys ? ep.row_sys[row0] : 0;
#pragma unroll
        for (int qa = 0; qa < MAXACC; ++qa) wq[qa] = (ep.row_sys && ep.coef_sys[qa]) ? ep.coef_sys[qa][sys] : ep.coef[qa];
    }
    const int4 *recs = reinterpret_cast<const int4 *>(plan.j_rec);
    const T *BtV = reinterpret_cast<const T *>(ops.bt_val);
    const T *Prev = reinterpret_cast<const T *>(ep.prev);
    const uint32_t *E32 = reinterpret_cast<const uint32_t *>(plan.entries);
    double tr = 0.0;

    // Column record (two int4): {j, Bt row start, Bt row length, first entry}
    // and {hit counts of rows 0..3 (8 bits each), out pos rows 0|1, 2|3, 0}.
    int4 ra = make_int4(-1, 0, 0, 0), rb = make_int4(0, -1, -1, 0);
    int4 raN = ra, rbN = rb;
    uint4 bt[RBV];
    uint32_t ew[kEntWords];
#define LREC(JJ, RA, RB)                                                              \
    do {                                                                              \
        if ((JJ) < nj) {                                                              \
            const i32x4 *r_ = reinterpret_cast<const i32x4 *>(recs) + 2 * (j0 + (JJ)); \
            const i32x4 a_ = ld_stream<NTH>(r_), b_ = ld_stream<NTH>(r_ + 1);          \
            RA = make_int4(a_.x, a_.y, a_.z, a_.w);                                   \
            RB = make_int4(b_.x, b_.y, b_.z, b_.w);                                   \
        } else {                                                                      \
            RA = make_int4(-1, 0, 0, 0);                                              \
        }                                                                             \
    } while (0)
// Row data of a column: uniform trip counts, no per-lane conditions (the
// buffers are padded so that reading up to one 64-lane round past the end is
// in bounds).
#define LROW(RA, RB, BT, EWD)                                                         \
    do {                                                                              \
        if ((RA).x >= 0) {                                                            \
            if (V16OK) {                                                              \
                const uint4 *src_ = reinterpret_cast<const uint4 *>(BtV + (int64_t)(RA).y * BB) + lane; \
                const int nv_ = ((RA).z * V16 + 63) >> 6;                             \
                _Pragma("unroll") for (int v_ = 0; v_ < RBV; ++v_)                    \
                    BT[v_] = (v_ < nv_) ? src_[v_ * 64] : make_uint4(0, 0, 0, 0);     \
            }                                                                         \
            const int tot_ = ((RB).x & 0xFF) + (((RB).x >> 8) & 0xFF) +               \
                             (((RB).x >> 16) & 0xFF) + (((RB).x >> 24) & 0xFF);        \
            const int nwv_ = ((tot_ * 2 * EW + 3) / 4 + 63) >> 6;                     \
            const uint32_t *es_ = E32 + ((int64_t)(RA).w * 2 * EW) / 4 + lane;        \
            _Pragma("unroll") for (int v_ = 0; v_ < kEntWords; ++v_)                  \
                EWD[v_] = (v_ < nwv_) ? ld_stream<NTH>(es_ + v_ * 64) : 0u;           \
        }                                                                             \
    } while (0)

    // epilogue operands of a column: output offsets and the values read back
    // (T_{k-1}, float64 accumulators)
#define LEPI(RA, RB, OFF, VAL, PRV, ACCV)                                             \
    do {                                                                              \
        _Pragma("unroll") for (int q_ = 0; q_ < NE; ++q_) {                           \
            unsigned op_ = 0xFFFFu;                                                   \
            int64_t cb_ = 0;                                                          \
            _Pragma("unroll") for (int i_ = 0; i_ < CMAX; ++i_) if (i_ == ei[q_]) {   \
                const uint32_t word_ = (i_ < 2) ? (uint32_t)(RB).y : (uint32_t)(RB).z; \
                op_ = (word_ >> ((i_ & 1) * 16)) & 0xFFFFu;                           \
                cb_ = cbase_i[i_];                                                    \
            }                                                                         \
            VAL[q_] = (RA).x >= 0 && ei[q_] < c && op_ != 0xFFFFu;                    \
            /* lanes without an output read element 0 and drop the value */          \
            OFF[q_] = VAL[q_] ? (cb_ + op_) * BB + er[q_] * B + es[q_] : 0;           \
            if (Prev) PRV[q_] = ld_stream<NTH>(Prev + OFF[q_]);                       \
            _Pragma("unroll") for (int qa_ = 0; qa_ < MAXACC; ++qa_)                  \
                if (qa_ < ep.nacc) ACCV[q_][qa_] = ld_stream<NTH>(ep.acc[qa_] + OFF[q_]); \
        }                                                                             \
    } while (0)

    // Software pipeline: every global load is issued one column before it is
    // used, in the order it is used (epilogue operands, Bt row and hit lists,
    // then the record of the column after), so that the in-order completion
    // of vector memory operations never makes a column wait for the loads of
    // the next one.
    // Two register sets used in turn (no copies between columns): the set of
    // column jj holds its record, Bt row, hit lists and epilogue operands; the
    // other set holds the record of column jj + NW.
    struct Set {
        int4 ra, rb;
        uint4 bt[RBV];
        uint32_t ew[kEntWords];
        int64_t off[NE];
        bool valid[NE];
        T prev[NE];
        double acc[NE][MAXACC];
    };
    Set S0, S1;
    S0.rb = make_int4(0, -1, -1, 0);
    S1.rb = S0.rb;
    auto column = [&](Set &C, Set &N, int JJ) __attribute__((always_inline)) {
        // loads for column JJ + NW (into N), then the record of JJ + 2 NW (into C)
        LEPI(N.ra, N.rb, N.off, N.valid, N.prev, N.acc);
        LROW(N.ra, N.rb, N.bt, N.ew);
        const int jc = C.ra.x, rowc = C.ra.y, nslc = C.ra.z, rbx = C.rb.x;
        (void)rowc;
        (void)nslc;
        LREC(JJ + 2 * NW, C.ra, C.rb);
        int cnt[CMAX], eoff[CMAX];
        {
            int acc_off = 0;
#pragma unroll
            for (int i = 0; i < CMAX; ++i) {
                cnt[i] = (rbx >> (8 * i)) & 0xFF;
                eoff[i] = acc_off;
                acc_off += cnt[i];
            }
        }
        // stage this column's Bt row and hit lists in the wave's LDS area
        const T *bsrc;
        if (V16OK) {
            uint4 *d16 = reinterpret_cast<uint4 *>(btw) + lane;
            const int nv = (nslc * V16 + 63) >> 6;
#pragma unroll
            for (int v = 0; v < RBV; ++v)
                if (v < nv) d16[v * 64] = C.bt[v];
            bsrc = btw;
        } else {
            bsrc = BtV + (int64_t)rowc * BB;
        }
        {
            uint32_t *e32 = reinterpret_cast<uint32_t *>(entw) + lane;
            const int tot = cnt[0] + (CMAX > 1 ? cnt[1 % CMAX] : 0) + (CMAX > 2 ? cnt[2 % CMAX] : 0) +
                            (CMAX > 3 ? cnt[3 % CMAX] : 0);
            const int nwv = ((tot * 2 * EW + 3) / 4 + 63) >> 6;
#pragma unroll
            for (int v = 0; v < kEntWords; ++v)
                if (v < nwv) e32[v * 64] = C.ew[v];
        }
        wave_sync_lds();

        T y[NE];
        if (MFMA) {
            // Branch-free loop: slots past the end of their row's list read the
            // zero block, so every lane issues the same instructions.
            const int mi = lane >> 4, grp = (lane >> 2) & 3, q = lane & 3;
            int nmax = 0, nmine = 0, omine = 0, rs = 0;
#pragma unroll
            for (int i = 0; i < CMAX; ++i) {
                nmax = max(nmax, cnt[i]);
                if (i == mi) {
                    nmine = cnt[i];
                    omine = eoff[i];
                    rs = rstart[i];
                }
            }
            nmax = __builtin_amdgcn_readfirstlane(nmax);
            typedef __attribute__((address_space(3))) const unsigned char lds_u8;
            typedef __attribute__((address_space(3))) const f32x4 lds_f4;
            // Bt operands: LDS (staged row) or global memory (BD)
            typedef typename std::conditional<BD, const unsigned char, lds_u8>::type b_u8;
            typedef typename std::conditional<BD, const f32x4, lds_f4>::type b_f4;
            lds_u8 *zp = (lds_u8 *)(As + (size_t)plan.lds_ablocks * BB);
            lds_u8 *a_base = (lds_u8 *)(As + rs * BB) + q * 16;
            b_u8 *b_base = (b_u8 *)bsrc + q * 16;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            const int iters = (nmax + 3) >> 2;
            // operand addresses of hit h of this slot (zero block past the list)
            // (past the end: A reads the zero block; B reads a block of the
            // row, finite, so the product is exactly zero)
            auto addr = [&](int hh, lds_u8 *&ap, b_u8 *&bp) {
                uint32_t pa, sl;
                // slots past their list read inside the wave's entry area
                // (the value is not used)
                const int ix = min(omine + hh, kEntMax - 1);
                if constexpr (EW == 1) {
                    const uint32_t e = reinterpret_cast<const uint16_t *>(entw)[ix];
                    pa = e & 0xFFu;
                    sl = e >> 8;
                } else {
                    const uint32_t e = reinterpret_cast<const uint32_t *>(entw)[ix];
                    pa = e & 0xFFFFu;
                    sl = e >> 16;
                }
                const bool ok = hh < nmine;
                ap = ok ? a_base + (pa << 6) : zp;
                if constexpr (BD)
                    bp = b_base + ((ok ? sl : 0u) << 6);
                else
                    bp = ok ? b_base + (sl << 6) : zp;
            };
            int it = 0;
            if constexpr (PIPE) {
                // groups of four hits per slot, software-pipelined: the
                // operands of group g + 1 are loaded while the MFMAs of group g
                // run (two register sets in turn); the remainder below
                auto load = [&](int g, f32x4 *a, f32x4 *bq) __attribute__((always_inline)) {
                    lds_u8 *ap[4];
                    b_u8 *bp[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) addr(grp + 4 * (4 * g + u), ap[u], bp[u]);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        a[u] = *(lds_f4 *)ap[u];
                        bq[u] = *(b_f4 *)bp[u];
                    }
                };
                auto mma = [&](const f32x4 *a, const f32x4 *bq, f32x4 &c) __attribute__((always_inline)) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        c = __builtin_amdgcn_mfma_f32_4x4x1f32(a[u][0], bq[u][0], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_4x4x1f32(a[u][1], bq[u][1], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_4x4x1f32(a[u][2], bq[u][2], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_4x4x1f32(a[u][3], bq[u][3], c, 0, 0, 0);
                    }
                };
                // Loads run one group ahead unconditionally (a group past the
                // list reads the zero block and slot 0: valid addresses, zero
                // products), so the wait before each group's MFMAs only covers
                // that group's loads; two accumulators keep consecutive MFMAs
                // independent.
                const int groups = iters >> 2;
                f32x4 a0[4], b0[4], a1[4], b1[4];
                f32x4 acc1 = {0.f, 0.f, 0.f, 0.f};
                load(0, a0, b0);
                for (int g = 0; g < groups; g += 2) {
                    load(g + 1, a1, b1);
                    mma(a0, b0, acc);
                    load(g + 2, a0, b0);
                    if (g + 1 < groups) mma(a1, b1, acc1);
                }
                acc += acc1;
                it = groups * 4;
            }
            // G hits per slot at a time: all operand loads issued before the
            // MFMAs (one wait per G hits); G > 4 alternates two accumulators
            if constexpr (G > 4) {
                f32x4 acc2 = {0.f, 0.f, 0.f, 0.f};
                // PAD: the last group runs past the lists (zero products), so a
                // column waits once per G hits and never in the loops below
                for (; PAD ? it < iters : it + G <= iters; it += G) {
                    lds_u8 *ap[G];
                    b_u8 *bp[G];
#pragma unroll
                    for (int u = 0; u < G; ++u) addr(grp + 4 * (it + u), ap[u], bp[u]);
                    f32x4 a[G], bb[G];
                    // keep every global load of the group ahead of its MFMAs
                    // (the scheduler would otherwise interleave them to save
                    // registers, leaving one or two loads in flight); with
                    // G > 6 the LDS reads of A follow the barrier, next to
                    // their MFMAs, to stay within 128 registers
#pragma unroll
                    for (int u = 0; u < G; ++u) {
                        if constexpr (G <= 6) a[u] = *(lds_f4 *)ap[u];
                        bb[u] = *(b_f4 *)bp[u];
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    if constexpr (G > 6) {
#pragma unroll
                        for (int u = 0; u < G; ++u) a[u] = *(lds_f4 *)ap[u];
                    }
#pragma unroll
                    for (int u = 0; u < G; ++u) {
                        f32x4 &c = (u & 1) ? acc2 : acc;
                        c = __builtin_amdgcn_mfma_f32_4x4x1f32(a[u][0], bb[u][0], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_4x4x1f32(a[u][1], bb[u][1], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_4x4x1f32(a[u][2], bb[u][2], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_4x4x1f32(a[u][3], bb[u][3], c, 0, 0, 0);
                    }
                }
                acc += acc2;
            }
            // four hits per slot at a time: all LDS reads issued before the MFMAs
            for (; it + 4 <= iters; it += 4) {
                lds_u8 *ap[4];
                b_u8 *bp[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) addr(grp + 4 * (it + u), ap[u], bp[u]);
                f32x4 a[4], bb[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a[u] = *(lds_f4 *)ap[u];
                    bb[u] = *(b_f4 *)bp[u];
                }
                if constexpr (SB) __builtin_amdgcn_sched_barrier(0);  // all loads before the MFMAs
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a[u][0], bb[u][0], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a[u][1], bb[u][1], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a[u][2], bb[u][2], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a[u][3], bb[u][3], acc, 0, 0, 0);
                }
            }
            for (; it < iters; ++it) {
                lds_u8 *ap;
                b_u8 *bp;
                addr(grp + 4 * it, ap, bp);
                const f32x4 a = *(lds_f4 *)ap;
                const f32x4 bb = *(b_f4 *)bp;
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
        } else if (MF64) {
            // v_mfma_f64_4x4x4f64 runs 4 independent 4x4x4 block products:
            // block blk = tile row; operand lane 16 t + 4 blk + x holds
            // A[blk][x][t] (row x of A[i, l], column t) and B[blk][t][x]
            // (= Bt[j, l][x][t]); one hit of every row per instruction, rows
            // past the end of their list read the zero block.
            const int blk = (lane >> 2) & 3;
            const int x = lane & 3, t = lane >> 4;
            int nmax = 0, nmine = 0, omine = 0, rs = 0;
#pragma unroll
            for (int i = 0; i < CMAX; ++i) {
                nmax = max(nmax, cnt[i]);
                if (i == blk) {
                    nmine = cnt[i];
                    omine = eoff[i];
                    rs = rstart[i];
                }
            }
            nmax = __builtin_amdgcn_readfirstlane(nmax);
            typedef __attribute__((address_space(3))) const unsigned char lds_u8;
            typedef __attribute__((address_space(3))) const double lds_d;
            typedef typename std::conditional<BD, const unsigned char, lds_u8>::type b_u8;
            typedef typename std::conditional<BD, const double, lds_d>::type b_d;
            lds_u8 *zp = (lds_u8 *)(As + (size_t)plan.lds_ablocks * BB);
            const int eoffb = (x * 4 + t) * 8;
            lds_u8 *a_base = (lds_u8 *)(As + rs * BB) + eoffb;
            b_u8 *b_base = (b_u8 *)bsrc + eoffb;
            double acc = 0.0;
            auto addr = [&](int hh, lds_u8 *&ap, b_u8 *&bp) {
                uint32_t pa, sl;
                // slots past their list read inside the wave's entry area
                // (the value is not used)
                const int ix = min(omine + hh, kEntMax - 1);
                if constexpr (EW == 1) {
                    const uint32_t e = reinterpret_cast<const uint16_t *>(entw)[ix];
                    pa = e & 0xFFu;
                    sl = e >> 8;
                } else {
                    const uint32_t e = reinterpret_cast<const uint32_t *>(entw)[ix];
                    pa = e & 0xFFFFu;
                    sl = e >> 16;
                }
                const bool ok = hh < nmine;
                ap = ok ? a_base + (pa << 7) : zp;
                if constexpr (BD)
                    bp = b_base + ((ok ? sl : 0u) << 7);
                else
                    bp = ok ? b_base + (sl << 7) : zp;
            };
            int h = 0;
            // with operands from global memory, 8 hits per wait (one MFMA
            // each) and two accumulators in turn
            if constexpr (BD) {
                double acc2 = 0.0;
                for (; h + 8 <= nmax; h += 8) {
                    lds_u8 *ap[8];
                    b_u8 *bp[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) addr(h + u, ap[u], bp[u]);
                    double a[8], bb[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        a[u] = *(lds_d *)ap[u];
                        bb[u] = *(b_d *)bp[u];
                    }
                    if constexpr (SB) __builtin_amdgcn_sched_barrier(0);  // all loads before the MFMAs
#pragma unroll
                    for (int u = 0; u < 8; u += 2) {
                        acc = __builtin_amdgcn_mfma_f64_4x4x4f64(a[u], bb[u], acc, 0, 0, 0);
                        acc2 = __builtin_amdgcn_mfma_f64_4x4x4f64(a[u + 1], bb[u + 1], acc2, 0, 0, 0);
                    }
                }
                acc += acc2;
            }
            for (; h + 4 <= nmax; h += 4) {
                lds_u8 *ap[4];
                b_u8 *bp[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) addr(h + u, ap[u], bp[u]);
                double a[4], bb[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a[u] = *(lds_d *)ap[u];
                    bb[u] = *(b_d *)bp[u];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_4x4x4f64(a[u], bb[u], acc, 0, 0, 0);
            }
            for (; h < nmax; ++h) {
                lds_u8 *ap;
                b_u8 *bp;
                addr(h, ap, bp);
                acc = __builtin_amdgcn_mfma_f64_4x4x4f64(*(lds_d *)ap, *(b_d *)bp, acc, 0, 0, 0);
            }
            y[0] = (T)acc;
        } else {
            int n[NE], o[NE], rsq[NE];
            int nmax = 0;
#pragma unroll
            for (int q = 0; q < NE; ++q) {
                n[q] = 0;
                o[q] = 0;
                rsq[q] = 0;
#pragma unroll
                for (int i = 0; i < CMAX; ++i)
                    if (i == ei[q]) {
                        n[q] = cnt[i];
                        o[q] = eoff[i];
                        rsq[q] = rstart[i];
                    }
                if (!C.valid[q]) n[q] = 0;
                nmax = max(nmax, n[q]);
                y[q] = (T)0;
            }
            for (int h = 0; h < nmax; ++h) {
#pragma unroll
                for (int q = 0; q < NE; ++q) {
                    if (h < n[q]) {
                        int pa, sl;
                        decode<EW>(entw, o[q] + h, pa, sl);
                        const T *a = As + (rsq[q] + pa) * BB + er[q] * B;
                        const T *bs = bsrc + (int64_t)sl * BB + es[q] * B;
                        T s = (T)0;
#pragma unroll
                        for (int t = 0; t < B; ++t) s = fma(a[t], bs[t], s);
                        y[q] += s;
                    }
                }
            }
        }
        // fused epilogue
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            if (!C.valid[q]) continue;
            T o = (T)ep.alpha * y[q];
            if (Prev) o = fma((T)ep.beta, C.prev[q], o);
            st_stream<NTH>(reinterpret_cast<T *>(ops.c_out) + C.off[q], o);
            const double od = (double)o;
#pragma unroll
            for (int qa = 0; qa < MAXACC; ++qa)
                if (qa < ep.nacc) st_stream<NTH>(ep.acc[qa] + C.off[q], C.acc[q][qa] + wq[qa] * od);
            if (ep.hist) st_stream<NTH>(reinterpret_cast<T *>(ep.hist) + C.off[q], o);
            if (row0 + ei[q] == jc && er[q] == es[q]) tr += od;
        }
        wave_sync_lds();
    };
    int jj = wave;
    LREC(jj, S0.ra, S0.rb);
    LEPI(S0.ra, S0.rb, S0.off, S0.valid, S0.prev, S0.acc);
    LROW(S0.ra, S0.rb, S0.bt, S0.ew);
    LREC(jj + NW, S1.ra, S1.rb);
    for (; jj < nj; jj += 2 * NW) {
        column(S0, S1, jj);
        if (jj + NW >= nj) break;
        column(S1, S0, jj + NW);
    }
#undef LEPI
#undef LREC
#undef LROW
    if (ep.trace_partial) {
        const double s = bsum<NT>(tr);
        if (threadIdx.x == 0) ep.trace_partial[tile] = s;
    }
}

// float32, b = 9, tiles of <= 2 rows, on v_mfma_f32_4x4x1f32: the 9 x 9
// output block of (row i, column j) is a 3 x 3 grid of 3 x 3 sub-blocks, one
// per MFMA slot (slots 0..8; lane q = 3 and slots 9..15 carry zeros).  Slot
// s = 3 I' + J' takes row 3 I' + q of A[i, l] as its A operand and row
// 3 J' + q of Bt[j, l] as its B operand, so nine MFMAs (k = 0..8) form one
// 9 x 9 x 9 block product; register v of lane (s, q) ends as element
// (3 I' + v, 3 J' + q).  Rows of the tile are taken one after the other;
// hit lists and the epilogue are those of k_listed.
template <int NW, int EW, int MAXACC>
__global__ __launch_bounds__(64 * NW) void k_listed9(ListedPlanDev plan, ProductOperands ops,
                                                     Epilogue ep) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    constexpr int BB = 81;
    constexpr int NT = 64 * NW;
    constexpr int kEntMax = kEntWords * 64 * 4 / (2 * EW);
    const int ntiles = plan.ntiles;
    const int nt8 = (ntiles + 7) & ~7;
    const int w = blockIdx.x;
    const int tile = (w & 7) * (nt8 >> 3) + (w >> 3);
    if (tile >= ntiles) return;
    const ListedLds L = listed_lds<float, 9, NW, EW, true>(plan);
    const int row0 = plan.tile_row0[tile];
    if (tile_finished(ep, tile, row0)) return;
    const int c = plan.tile_row0[tile + 1] - row0;
    const int64_t ab0 = ops.a_rp[row0];
    float *As = reinterpret_cast<float *>(smem + L.a);
    {
        const int nab = (int)(ops.a_rp[row0 + c] - ab0);
        const float *Ag = reinterpret_cast<const float *>(ops.a_val) + ab0 * BB;
        for (int x = threadIdx.x; x < nab * BB; x += NT) As[x] = Ag[x];
        for (int x = threadIdx.x; x < BB; x += NT) As[(size_t)plan.lds_ablocks * BB + x] = 0.f;
    }
    int rstart[2];
    int64_t cbase_i[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        rstart[i] = (i < c) ? (int)(ops.a_rp[row0 + i] - ab0) : 0;
        cbase_i[i] = (i < c) ? ops.c_rp[row0 + i] : 0;
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    unsigned char *entw = smem + L.wave + (size_t)wave * (L.wave_bt + L.wave_ent) + L.wave_bt;
    const int slot = lane >> 2, q = lane & 3;
    const bool live = slot < 9 && q < 3;
    const int arow = 3 * (slot / 3) + q, bcol = 3 * (slot % 3) + q;
    typedef __attribute__((address_space(3))) const float lds_f;
    lds_f *zrow = (lds_f *)(As + (size_t)plan.lds_ablocks * BB);
    const int64_t j0 = plan.j_off[tile];
    const int nj = (int)(plan.j_off[tile + 1] - j0);
    const int4 *recs = reinterpret_cast<const int4 *>(plan.j_rec);
    const float *BtV = reinterpret_cast<const float *>(ops.bt_val);
    const float *Prev = reinterpret_cast<const float *>(ep.prev);
    const uint32_t *E32 = reinterpret_cast<const uint32_t *>(plan.entries);
    double wq[MAXACC];
    {
        const int sys = ep.row_sys ? ep.row_sys[row0] : 0;
#pragma unroll
        for (int qa = 0; qa < MAXACC; ++qa) wq[qa] = (ep.row_sys && ep.coef_sys[qa]) ? ep.coef_sys[qa][sys] : ep.coef[qa];
    }
    double tr = 0.0;
    for (int jj = wave; jj < nj; jj += NW) {
        const int4 ra = recs[2 * (j0 + jj)], rb = recs[2 * (j0 + jj) + 1];
        const int jc = ra.x, rowc = ra.y;
        int cnt[2], eoff[2];
        cnt[0] = rb.x & 0xFF;
        cnt[1] = (rb.x >> 8) & 0xFF;
        eoff[0] = 0;
        eoff[1] = cnt[0];
        {
            // this column's hit lists -> the wave's LDS area
            const int tot = cnt[0] + cnt[1];
            const int nwv = ((tot * 2 * EW + 3) / 4 + 63) >> 6;
            const uint32_t *es = E32 + ((int64_t)ra.w * 2 * EW) / 4 + lane;
            uint32_t *e32 = reinterpret_cast<uint32_t *>(entw) + lane;
#pragma unroll
            for (int v = 0; v < kEntWords; ++v)
                if (v < nwv) e32[v * 64] = es[v * 64];
        }
        wave_sync_lds();
        const float *bbase = BtV + (int64_t)rowc * BB + (live ? bcol : 0) * 9;
        for (int i = 0; i < c; ++i) {
            const uint32_t word = (uint32_t)rb.y;
            const unsigned op = (word >> (i * 16)) & 0xFFFFu;
            if (op == 0xFFFFu) continue;  // (i, j) not in the output pattern
            f32x4 acc = {0.f, 0.f, 0.f, 0.f}, acc2 = {0.f, 0.f, 0.f, 0.f};
            lds_f *abase = (lds_f *)(As + (size_t)rstart[i] * BB + arow * 9);
            const int n = cnt[i];
            for (int h = 0; h < n; h += 2) {
                // two hits per wait (the second past the list reads zeros)
                float a0[9], b0[9], a1[9], b1[9];
                int pa0, sl0, pa1, sl1;
                decode<EW>(entw, min(eoff[i] + h, kEntMax - 1), pa0, sl0);
                decode<EW>(entw, min(eoff[i] + h + 1, kEntMax - 1), pa1, sl1);
                const bool ok1 = h + 1 < n;
                lds_f *ap0 = live ? abase + pa0 * BB : zrow;
                lds_f *ap1 = (live && ok1) ? abase + pa1 * BB : zrow;
                const float *bp0 = bbase + (int64_t)sl0 * BB;
                const float *bp1 = bbase + (int64_t)(ok1 ? sl1 : sl0) * BB;
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    a0[k] = ap0[k];
                    b0[k] = bp0[k];
                    a1[k] = ap1[k];
                    b1[k] = bp1[k];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a0[k], b0[k], acc, 0, 0, 0);
                    acc2 = __builtin_amdgcn_mfma_f32_4x4x1f32(a1[k], b1[k], acc2, 0, 0, 0);
                }
            }
            acc += acc2;
            if (live) {
#pragma unroll
                for (int v = 0; v < 3; ++v) {
                    const int r = 3 * (slot / 3) + v, cc = bcol;
                    const int64_t off = (cbase_i[i] + op) * BB + r * 9 + cc;
                    float o = (float)ep.alpha * acc[v];
                    if (Prev) o = fmaf((float)ep.beta, Prev[off], o);
                    reinterpret_cast<float *>(ops.c_out)[off] = o;
                    const double od = (double)o;
#pragma unroll
                    for (int qa = 0; qa < MAXACC; ++qa)
                        if (qa < ep.nacc) ep.acc[qa][off] = ep.acc[qa][off] + wq[qa] * od;
                    if (ep.hist) reinterpret_cast<float *>(ep.hist)[off] = o;
                    if (row0 + i == jc && r == cc) tr += od;
                }
            }
        }
        wave_sync_lds();
    }
    if (ep.trace_partial) {
        const double sm = bsum<NT>(tr);
        if (threadIdx.x == 0) ep.trace_partial[tile] = sm;
    }
}

template <int NW, int EW, int MAXACC>
hipError_t launch_9(const ListedPlanDev &plan, const ProductOperands &ops, const Epilogue &ep,
                    hipStream_t st, size_t *lds_out) {
    const size_t lds = listed_lds<float, 9, NW, EW, true>(plan).total;
    if (lds_out) {
        *lds_out = lds;
        return hipSuccess;
    }
    if (plan.ntiles == 0) return hipSuccess;
    const void *fn = (const void *)k_listed9<NW, EW, MAXACC>;
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
    hipLaunchKernelGGL((k_listed9<NW, EW, MAXACC>), dim3(nt8), dim3(64 * NW), lds, st, plan, ops, ep);
    return hipGetLastError();
}

// float32, b = 4, tiles of <= 4 rows, on v_mfma_f32_4x4x1f32 with the 16 MFMA
// slots shared freely among the tile rows (plan.lean_rec / lean_ent).  With
// four slots fixed per row (k_listed) a column costs max_i ceil(cnt_i / 4)
// rounds of all 16 slots, so short or absent rows leave slots idle; here the
// host gives row i n_i consecutive slots (sum <= 16) so that the rounds
// R = max_i ceil(cnt_i / n_i) are as few as possible, and lays the hits out
// per round as 16 one-byte positions in the A rows, then 16 in the Bt row.
// A slot past its list reads its row's first A block and Bt position 255,
// outside the row: the buffer load returns zeros there, so the padded
// products add exact zeros and the loop has no per-hit conditions.  Each lane
// needs two LDS byte reads and two address operations per hit.  After the
// rounds the slots' partial blocks go to the wave's LDS area and each output
// lane sums those of its row's slots.  Groups of GM rounds issue all loads
// before their MFMAs (one wait per group); prefetching of records, hit lists
// and epilogue operands one column ahead and the epilogue follow k_listed.
struct LeanLds {
    size_t a, rec, wave, total;
};

// k_lean LDS: the A tile, the tile's column records, then 1 KB per wave (hit
// lists of the column, then the slots' partial blocks)
template <int NW>
__host__ __device__ inline LeanLds lean_lds(const ListedPlanDev &p) {
    LeanLds L;
    L.a = 0;
    L.rec = al16((size_t)p.lds_ablocks * 64);
    L.wave = L.rec + al16((size_t)p.max_cols * 32);
    L.total = L.wave + (size_t)NW * 1024;
    return L;
}

// (10 waves: two workgroups per CU need 5 waves per SIMD, at most 96 VGPRs)
template <int NW, int GM, bool LATE, int MAXACC>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW == 10 ? 5 : 1)))
void k_lean(ListedPlanDev plan, ProductOperands ops, Epilogue ep) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    constexpr int NT = 64 * NW;
    static_assert(GM == 4 || GM == 8, "rounds per group");
    const int ntiles = plan.ntiles;
    const int nt8 = (ntiles + 7) & ~7;
    const int w = blockIdx.x;
    const int tile = (w & 7) * (nt8 >> 3) + (w >> 3);
    if (tile >= ntiles) return;
    const LeanLds L = lean_lds<NW>(plan);
    const int row0 = plan.tile_row0[tile];
    if (tile_finished(ep, tile, row0)) return;
    const int c = plan.tile_row0[tile + 1] - row0;
    const int64_t ab0 = ops.a_rp[row0];
    const int64_t j0 = plan.j_off[tile];
    const int nj = (int)(plan.j_off[tile + 1] - j0);
    float *As = reinterpret_cast<float *>(smem + L.a);
    {
        // tile rows of A and the tile's column records -> LDS (records in
        // LDS keep their loads out of the in-order vector memory queue)
        const int n16 = (int)(ops.a_rp[row0 + c] - ab0) * 4;
        const u32x4 *src = reinterpret_cast<const u32x4 *>(reinterpret_cast<const float *>(ops.a_val) + ab0 * 16);
        u32x4 *dst = reinterpret_cast<u32x4 *>(As);
        for (int x = threadIdx.x; x < n16; x += NT) dst[x] = src[x];
        const i32x4 *rsrc = reinterpret_cast<const i32x4 *>(plan.lean_rec) + 2 * j0;
        i32x4 *rdst = reinterpret_cast<i32x4 *>(smem + L.rec);
        for (int x = threadIdx.x; x < 2 * nj; x += NT) rdst[x] = rsrc[x];
    }
    // first A block of each tile row in the LDS tile (named values, not an
    // array: a per-lane index into an array would go through scratch memory)
    const int rs0 = 0;
    const int rs1 = (1 < c) ? (int)(ops.a_rp[row0 + 1] - ab0) : 0;
    const int rs2 = (2 < c) ? (int)(ops.a_rp[row0 + 2] - ab0) : 0;
    const int rs3 = (3 < c) ? (int)(ops.a_rp[row0 + 3] - ab0) : 0;
    __syncthreads();

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    unsigned char *entw = smem + L.wave + (size_t)wave * 1024;
    // MFMA operand lane: slot and row q of its blocks; output lane: element
    // (er, es) of tile row oi
    const int slot = lane >> 2, q = lane & 3;
    const int oi = lane >> 4, er = (lane >> 2) & 3, es = lane & 3;
    // first output element of this lane's row (element offsets of the
    // kernel pattern fit in 31 bits: checked when the plan is built)
    const uint32_t cb_mine = (oi < c) ? (uint32_t)ops.c_rp[row0 + oi] * 16u + er * 4 + es : 0u;
    double wq[MAXACC > 0 ? MAXACC : 1];
    {
        const int sys = ep.row_sys ? ep.row_sys[row0] : 0;
#pragma unroll
        for (int qa = 0; qa < MAXACC; ++qa) wq[qa] = (ep.row_sys && ep.coef_sys[qa]) ? ep.coef_sys[qa][sys] : ep.coef[qa];
    }
    typedef __attribute__((address_space(3))) const i32x4 lds_i4;
    const lds_i4 *recs = (const lds_i4 *)(smem + L.rec);
    const float *BtV = reinterpret_cast<const float *>(ops.bt_val);
    const float *Prev = reinterpret_cast<const float *>(ep.prev);
    double tr = 0.0;
    typedef __attribute__((address_space(3))) const unsigned char lds_u8;
    typedef __attribute__((address_space(3))) const f32x4 lds_f4;

    // The prefetch loads below are unconditional (past the last column they
    // re-read the last record; unused words of a hit list re-read its first
    // word; a missing T_{k-1} reads T_k, a missing sum the first one), so
    // that no branch joins make the compiler wait for them early.
    // Streamed operands go through buffer descriptors (32-bit offsets, one
    // VGPR per address instead of a 64-bit pointer)
    constexpr int kAll = 0x7FFFFFFF;
    auto rsrc = [](const void *p) __attribute__((always_inline)) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, kAll, 0x00020000);
    };
    const __amdgpu_buffer_rsrc_t r_prev = rsrc(Prev ? ep.prev : ops.a_val);
    const __amdgpu_buffer_rsrc_t r_out = rsrc(ops.c_out);
    const __amdgpu_buffer_rsrc_t r_hist = rsrc(ep.hist ? ep.hist : ops.c_out);
    const __amdgpu_buffer_rsrc_t r_ent = rsrc(plan.lean_ent);
    constexpr int NACC = MAXACC > 0 ? MAXACC : 1;
    __amdgpu_buffer_rsrc_t r_acc[NACC];
#pragma unroll
    for (int qa = 0; qa < NACC; ++qa) r_acc[qa] = rsrc((qa < ep.nacc) ? ep.acc[qa] : ep.acc[0]);
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    struct Set {
        i32x4 ra, rb;
        uint32_t ew[kEntWords];
        uint32_t off;
        bool live, valid;
        float prev;
        double acc[NACC];
    };
    // record of column JJ (nj >= 1)
    auto lrec = [&](int JJ, Set &S) __attribute__((always_inline)) {
        const int jl = min(JJ, nj - 1);
        S.ra = recs[2 * jl];
        S.rb = recs[2 * jl + 1];
        S.live = JJ < nj;
    };
    // hit lists (R rounds of 32 bytes, at most 1 KB), then the epilogue
    // operands of the column in S
    auto lrow = [&](Set &S) __attribute__((always_inline)) {
        const int rbx = __builtin_amdgcn_readfirstlane(S.rb.x);
        const int first = __builtin_amdgcn_readfirstlane(S.ra.w);
        const int nwv = S.live ? ((rbx & 0xFF) * 8 + 63) >> 6 : 0;
#pragma unroll
        for (int v = 0; v < kEntWords; ++v)
            S.ew[v] = __builtin_amdgcn_raw_buffer_load_b32(r_ent, lane * 4, first * 32 + (v < nwv ? v * 256 : 0), 0);
        const uint32_t word = (oi < 2) ? (uint32_t)S.rb.y : (uint32_t)S.rb.z;
        const unsigned op = (word >> ((oi & 1) * 16)) & 0xFFFFu;
        S.valid = S.live && oi < c && op != 0xFFFFu;
        // lanes without an output read element 0 and drop the value
        S.off = S.valid ? cb_mine + op * 16u : 0u;
        S.prev = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r_prev, (int)(S.off * 4), 0, 0));
#pragma unroll
        for (int qa = 0; qa < MAXACC; ++qa)
            S.acc[qa] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r_acc[qa], (int)(S.off * 8), 0, 0));
    };

    auto column = [&](Set &C, Set &N, int JJ) __attribute__((always_inline)) {
        const int jc = C.ra.x;
        const int rowc = __builtin_amdgcn_readfirstlane(C.ra.y);
        const int lenc = __builtin_amdgcn_readfirstlane(C.ra.z);
        const int rbx = __builtin_amdgcn_readfirstlane(C.rb.x);
        // loads for column JJ + NW (into N), then the record of JJ + 2 NW
        // (into C).  Vector memory loads complete in order, so every wait for
        // a group's Bt operands also waits for all loads issued before them:
        // LATE issues these after the Bt loads of the column's last group,
        // so that they overlap that group's MFMAs, the row sums and the
        // epilogue instead of delaying the column's first MFMA
        auto prefetch = [&]() __attribute__((always_inline)) {
            lrow(N);
            lrec(JJ + 2 * NW, C);
        };
        if constexpr (!LATE) prefetch();
        const int R = rbx & 0xFF;
        {
            // all four words (the area is 1 KB): no branches, no early waits
            uint32_t *e32 = reinterpret_cast<uint32_t *>(entw) + lane;
#pragma unroll
            for (int v = 0; v < kEntWords; ++v) e32[v * 64] = C.ew[v];
        }
        wave_sync_lds();
        const int n0 = (rbx >> 8) & 31, n1 = (rbx >> 13) & 31, n2 = (rbx >> 18) & 31, n3 = (rbx >> 23) & 31;
        const int p1 = n0, p2 = p1 + n1, p3 = p2 + n2;
        // first A block of this slot's row (slots past the last row's take
        // row 3's, which is in the tile)
        const int rs = slot >= p3 ? rs3 : slot >= p2 ? rs2 : slot >= p1 ? rs1 : rs0;
        lds_u8 *a_base = (lds_u8 *)As + rs * 64 + q * 16;
        lds_u8 *e_base = (lds_u8 *)entw + slot;
        const __amdgpu_buffer_rsrc_t brs =
            __builtin_amdgcn_make_buffer_rsrc((void *)(BtV + (int64_t)rowc * 16), (short)0, lenc * 64, 0x00020000);
        const int boff = q * 16;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f}, acc2 = {0.f, 0.f, 0.f, 0.f};
        auto group = [&](auto gg, auto hook, int r0) __attribute__((always_inline)) {
            constexpr int GG = decltype(gg)::value;
            constexpr bool HOOK = decltype(hook)::value;
            lds_u8 *e0 = e_base + r0 * 32;
            uint32_t av[GG], bv[GG];
#pragma unroll
            for (int u = 0; u < GG; ++u) {
                av[u] = e0[u * 32];
                bv[u] = e0[u * 32 + 16];
            }
            u32x4 bb[GG];
            f32x4 a[GG];
#pragma unroll
            for (int u = 0; u < GG; ++u) {
                bb[u] = __builtin_amdgcn_raw_buffer_load_b128(brs, (int)((bv[u] << 6) + boff), 0, 0);
                if constexpr (GG <= 4) a[u] = *(lds_f4 *)(a_base + (av[u] << 6));
            }
            if constexpr (HOOK) prefetch();
            // every global load of the group ahead of its MFMAs; with 8
            // rounds the LDS reads of A follow, next to their MFMAs
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (GG > 4) {
#pragma unroll
                for (int u = 0; u < GG; ++u) a[u] = *(lds_f4 *)(a_base + (av[u] << 6));
            }
#pragma unroll
            for (int u = 0; u < GG; ++u) {
                f32x4 &cc = (u & 1) ? acc2 : acc;
                const f32x4 b = __builtin_bit_cast(f32x4, bb[u]);
                cc = __builtin_amdgcn_mfma_f32_4x4x1f32(a[u][0], b[0], cc, 0, 0, 0);
                cc = __builtin_amdgcn_mfma_f32_4x4x1f32(a[u][1], b[1], cc, 0, 0, 0);
                cc = __builtin_amdgcn_mfma_f32_4x4x1f32(a[u][2], b[2], cc, 0, 0, 0);
                cc = __builtin_amdgcn_mfma_f32_4x4x1f32(a[u][3], b[3], cc, 0, 0, 0);
            }
        };
        // R (even) = GM m + t: m groups of GM rounds, then 4 (if t & 4, GM = 8)
        // and 2 (if t & 2); LATE: the prefetch goes with the last group
        using G2 = std::integral_constant<int, 2>;
        using G4 = std::integral_constant<int, 4>;
        using GF = std::integral_constant<int, GM>;
        using NOH = std::integral_constant<bool, false>;
        using LH = std::integral_constant<bool, LATE>;
        const int m = R / GM, t = R % GM;
        const bool has4 = GM > 4 && (t & 4) != 0, has2 = (t & 2) != 0;
        const int mlast = (has4 || has2 || m == 0) ? m : m - 1;  // plain full groups
        int r = 0;
        for (int g = 0; g < mlast; ++g, r += GM) group(GF{}, NOH{}, r);
        if (!has4 && !has2) {
            if (m > 0) {
                group(GF{}, LH{}, r);
            } else if constexpr (LATE) {
                prefetch();
            }
        } else {
            if constexpr (GM > 4) {
                if (has4) {
                    if (has2) {
                        group(G4{}, NOH{}, r);
                    } else {
                        group(G4{}, LH{}, r);
                    }
                    r += 4;
                }
            }
            if (has2) group(G2{}, LH{}, r);
        }
        acc += acc2;
        // partial block of each slot -> LDS (element (v, q) of slot s at
        // float s * 16 + q * 4 + v); the hit lists there have been read
        reinterpret_cast<f32x4 *>(entw)[lane] = acc;
        wave_sync_lds();
        const float *pl = reinterpret_cast<const float *>(entw);
        int so = 0, no = n0;
        if (oi == 1) { so = p1; no = n1; }
        if (oi == 2) { so = p2; no = n2; }
        if (oi == 3) { so = p3; no = n3; }
        float y = 0.f;
        {
            const float *pk = pl + so * 16 + es * 4 + er;
            for (int k = 0; k < no; ++k) y += pk[k * 16];
        }
        wave_sync_lds();  // the area takes the next column's lists
        // fused epilogue
        if (C.valid) {
            float o = (float)ep.alpha * y;
            if (Prev) o = fmaf((float)ep.beta, C.prev, o);
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, o), r_out, (int)(C.off * 4), 0, 0);
            const double od = (double)o;
#pragma unroll
            for (int qa = 0; qa < MAXACC; ++qa)
                if (qa < ep.nacc)
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, C.acc[qa] + wq[qa] * od), r_acc[qa],
                                                          (int)(C.off * 8), 0, 0);
            if (ep.hist) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, o), r_hist, (int)(C.off * 4), 0, 0);
            if (row0 + oi == jc && er == es) tr += od;
        }
    };
    if (nj > 0) {
        Set S0, S1;
        int jj = wave;
        lrec(jj, S0);
        lrow(S0);
        lrec(jj + NW, S1);
        for (; jj < nj; jj += 2 * NW) {
            column(S0, S1, jj);
            if (jj + NW >= nj) break;
            column(S1, S0, jj + NW);
        }
    }
    if (ep.trace_partial) {
        const double s = bsum<NT>(tr);
        if (threadIdx.x == 0) ep.trace_partial[tile] = s;
    }
}

template <int NW, int GM, bool LATE, int MAXACC>
hipError_t launch_lean_a(const ListedPlanDev &plan, const ProductOperands &ops, const Epilogue &ep,
                         hipStream_t st, size_t *lds_out) {
    const size_t lds = lean_lds<NW>(plan).total;
    if (lds_out) {
        *lds_out = lds;
        return hipSuccess;
    }
    if (plan.ntiles == 0) return hipSuccess;
    if (!plan.lean_rec || plan.entry_width != 1 || plan.cmax != 4) return hipErrorInvalidValue;
    const void *fn = (const void *)k_lean<NW, GM, LATE, MAXACC>;
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
    hipLaunchKernelGGL((k_lean<NW, GM, LATE, MAXACC>), dim3(nt8), dim3(64 * NW), lds, st, plan, ops, ep);
    return hipGetLastError();
}

template <int NW, int GM, bool LATE = false>
hipError_t launch_lean(const ListedPlanDev &plan, const ProductOperands &ops, const Epilogue &ep,
                       hipStream_t st, size_t *lds_out) {
    if (ep.nacc <= 0) return launch_lean_a<NW, GM, LATE, 0>(plan, ops, ep, st, lds_out);
    if (ep.nacc == 1) return launch_lean_a<NW, GM, LATE, 1>(plan, ops, ep, st, lds_out);
    return launch_lean_a<NW, GM, LATE, 4>(plan, ops, ep, st, lds_out);
}

struct Lean9Lds {
    size_t a, rec, wave, total;
};

// k_lean9 LDS: the A tile and a zero block, the tile's column records, then
// 1 KB per wave for the column's hit lists
template <int NW>
__host__ __device__ inline Lean9Lds lean9_lds(const ListedPlanDev &p) {
    Lean9Lds L;
    L.a = 0;
    L.rec = al16((size_t)(p.lds_ablocks + 1) * 81 * sizeof(float));
    L.wave = L.rec + al16((size_t)p.max_cols * 32);
    L.total = L.wave + (size_t)NW * 1024;
    return L;
}

// float32, b = 9, tiles of <= 2 rows: the MFMA block mapping of k_listed9
// with the column pipelining of k_lean.  The tile's column records are copied
// to LDS with the A tile; the hit lists and the epilogue operands of the next
// column are loaded without branches, after the Bt loads of the column's last
// hit group (vector memory loads complete in order, so loads issued earlier
// would delay that group's MFMAs); Bt, hit lists and epilogue operands go
// through buffer descriptors.  MAXACC 0 or 1: no sum, or one sum whose
// operands are prefetched with the column's; MAXACC 4: up to four sums
// (batches, matrix powers with two exponents), each read in the column's
// epilogue, so that the pipelined state holds no sums.
template <int NW, int MAXACC>
__global__ __launch_bounds__(64 * NW) void k_lean9(ListedPlanDev plan, ProductOperands ops, Epilogue ep) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    constexpr int BB = 81;
    constexpr int NT = 64 * NW;
    constexpr int kEntMax = kEntWords * 64 * 2;  // 2-byte entries in a wave's 1 KB
    static_assert(MAXACC == 0 || MAXACC == 1 || MAXACC == 4, "zero, one or up to four float64 sums");
    const int ntiles = plan.ntiles;
    const int nt8 = (ntiles + 7) & ~7;
    const int w = blockIdx.x;
    const int tile = (w & 7) * (nt8 >> 3) + (w >> 3);
    if (tile >= ntiles) return;
    const Lean9Lds L = lean9_lds<NW>(plan);
    const int row0 = plan.tile_row0[tile];
    if (tile_finished(ep, tile, row0)) return;
    const int c = plan.tile_row0[tile + 1] - row0;
    const int64_t ab0 = ops.a_rp[row0];
    const int64_t j0 = plan.j_off[tile];
    const int nj = (int)(plan.j_off[tile + 1] - j0);
    float *As = reinterpret_cast<float *>(smem + L.a);
    {
        const int nab = (int)(ops.a_rp[row0 + c] - ab0);
        const float *Ag = reinterpret_cast<const float *>(ops.a_val) + ab0 * BB;
        for (int x = threadIdx.x; x < nab * BB; x += NT) As[x] = Ag[x];
        for (int x = threadIdx.x; x < BB; x += NT) As[(size_t)plan.lds_ablocks * BB + x] = 0.f;
        const i32x4 *rsrc = reinterpret_cast<const i32x4 *>(plan.j_rec) + 2 * j0;
        i32x4 *rdst = reinterpret_cast<i32x4 *>(smem + L.rec);
        for (int x = threadIdx.x; x < 2 * nj; x += NT) rdst[x] = rsrc[x];
    }
    const int rs1 = (1 < c) ? (int)(ops.a_rp[row0 + 1] - ab0) : 0;
    // element offsets of the kernel pattern fit in 31 bits (checked on the host)
    const uint32_t cb0 = (uint32_t)ops.c_rp[row0];
    const uint32_t cb1 = (1 < c) ? (uint32_t)ops.c_rp[row0 + 1] : 0u;
    __syncthreads();

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    unsigned char *entw = smem + L.wave + (size_t)wave * 1024;
    const int slot = lane >> 2, q = lane & 3;
    const bool live = slot < 9 && q < 3;
    const int arow = 3 * (slot / 3) + q, bcol = 3 * (slot % 3) + q;
    typedef __attribute__((address_space(3))) const float lds_f;
    typedef __attribute__((address_space(3))) const i32x4 lds_i4;
    lds_f *zrow = (lds_f *)(As + (size_t)plan.lds_ablocks * BB);
    lds_f *abase0 = (lds_f *)(As + arow * 9);
    lds_f *abase1 = (lds_f *)(As + (size_t)rs1 * BB + arow * 9);
    const lds_i4 *recs = (const lds_i4 *)(smem + L.rec);
    // this lane's three outputs of a block: rows 3 (slot / 3) + v, column bcol
    const uint32_t eo = (uint32_t)(3 * (slot / 3) * 9 + bcol);
    const float *BtV = reinterpret_cast<const float *>(ops.bt_val);
    const float *Prev = reinterpret_cast<const float *>(ep.prev);
    double wq[4] = {0.0, 0.0, 0.0, 0.0};
    if (MAXACC > 0) {
        const int sys = ep.row_sys ? ep.row_sys[row0] : 0;
#pragma unroll
        for (int qa = 0; qa < MAXACC; ++qa)
            wq[qa] = (ep.row_sys && ep.coef_sys[qa]) ? ep.coef_sys[qa][sys] : ep.coef[qa];
    }
    constexpr int kAll = 0x7FFFFFFF;
    auto rsrc = [](const void *p, int n) __attribute__((always_inline)) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, n, 0x00020000);
    };
    const __amdgpu_buffer_rsrc_t r_prev = rsrc(Prev ? ep.prev : ops.a_val, kAll);
    const __amdgpu_buffer_rsrc_t r_out = rsrc(ops.c_out, kAll);
    const __amdgpu_buffer_rsrc_t r_hist = rsrc(ep.hist ? ep.hist : ops.c_out, kAll);
    __amdgpu_buffer_rsrc_t r_acc[MAXACC > 0 ? MAXACC : 1];
#pragma unroll
    for (int qa = 0; qa < (MAXACC > 0 ? MAXACC : 1); ++qa)
        r_acc[qa] = rsrc((MAXACC > 0 && qa < ep.nacc) ? (const void *)ep.acc[qa] : ops.c_out, kAll);
    const __amdgpu_buffer_rsrc_t r_ent = rsrc(plan.entries, kAll);
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    constexpr int NA = MAXACC == 1 ? 1 : 0;  // sums prefetched with the column
    struct Set {
        i32x4 ra, rb;
        uint32_t ew[kEntWords];
        uint32_t off[2];
        bool live, val[2];
        float prev[2][3];
        double acc[2][3 * NA + 1 - NA];
    };
    auto lrec = [&](int JJ, Set &S) __attribute__((always_inline)) {
        const int jl = min(JJ, nj - 1);
        S.ra = recs[2 * jl];
        S.rb = recs[2 * jl + 1];
        S.live = JJ < nj;
    };
    // hit lists, then the epilogue operands (unconditional loads: past the
    // last column the last record, unused words the first one, lanes
    // without an output element 0)
    auto lrow = [&](Set &S) __attribute__((always_inline)) {
        const int rbx = __builtin_amdgcn_readfirstlane(S.rb.x);
        const int first = __builtin_amdgcn_readfirstlane(S.ra.w);
        const int tot = (rbx & 0xFF) + ((rbx >> 8) & 0xFF);
        const int nwv = S.live ? ((tot * 2 + 3) / 4 + 63) >> 6 : 0;
#pragma unroll
        for (int v = 0; v < kEntWords; ++v)
            S.ew[v] = __builtin_amdgcn_raw_buffer_load_b32(r_ent, lane * 4, first * 2 + (v < nwv ? v * 256 : 0), 0);
        const uint32_t word = (uint32_t)S.rb.y;
        const uint32_t op0 = word & 0xFFFFu, op1 = word >> 16;
        S.val[0] = S.live && live && op0 != 0xFFFFu;
        S.val[1] = S.live && live && 1 < c && op1 != 0xFFFFu;
        S.off[0] = S.val[0] ? (cb0 + op0) * 81u + eo : 0u;
        S.off[1] = S.val[1] ? (cb1 + op1) * 81u + eo : 0u;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                const uint32_t e = S.off[i] + v * 9;
                S.prev[i][v] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r_prev, (int)(e * 4), 0, 0));
                if constexpr (MAXACC == 1)
                    S.acc[i][v] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r_acc[0], (int)(e * 8), 0, 0));
            }
    };
    double tr = 0.0;
    auto column = [&](Set &C, Set &N, int JJ) __attribute__((always_inline)) {
        const int jc = C.ra.x;
        const int rowc = __builtin_amdgcn_readfirstlane(C.ra.y);
        const int lenc = __builtin_amdgcn_readfirstlane(C.ra.z);
        const int rbx = __builtin_amdgcn_readfirstlane(C.rb.x);
        auto prefetch = [&]() __attribute__((always_inline)) {
            lrow(N);
            lrec(JJ + 2 * NW, C);
        };
        const int cnt0 = rbx & 0xFF, cnt1 = (rbx >> 8) & 0xFF;
        {
            uint32_t *e32 = reinterpret_cast<uint32_t *>(entw) + lane;
#pragma unroll
            for (int v = 0; v < kEntWords; ++v) e32[v * 64] = C.ew[v];
        }
        wave_sync_lds();
        const __amdgpu_buffer_rsrc_t brs = rsrc(BtV + (int64_t)rowc * BB, lenc * BB * 4);
        const int boff = bcol * 36;
        f32x4 a0 = {0.f, 0.f, 0.f, 0.f}, a0b = a0, a1 = a0, a1b = a0;
        // two hits of one row per wait (the second past the list reads zeros)
        auto grp = [&](auto ri, auto hook, int h) __attribute__((always_inline)) {
            constexpr int RI = decltype(ri)::value;
            constexpr bool HOOK = decltype(hook)::value;
            const int n = RI ? cnt1 : cnt0;
            const int eoff = RI ? cnt0 : 0;
            lds_f *abase = RI ? abase1 : abase0;
            f32x4 &acc = RI ? a1 : a0;
            f32x4 &acc2 = RI ? a1b : a0b;
            int pa0, sl0, pa1, sl1;
            decode<1>(entw, min(eoff + h, kEntMax - 1), pa0, sl0);
            decode<1>(entw, min(eoff + h + 1, kEntMax - 1), pa1, sl1);
            const bool ok1 = h + 1 < n;
            lds_f *ap0 = live ? abase + pa0 * BB : zrow;
            lds_f *ap1 = (live && ok1) ? abase + pa1 * BB : zrow;
            const int vo0 = sl0 * (BB * 4) + boff, vo1 = (ok1 ? sl1 : sl0) * (BB * 4) + boff;
            float x0[9], y0[9], x1[9], y1[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                y0[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(brs, vo0 + 4 * k, 0, 0));
                y1[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(brs, vo1 + 4 * k, 0, 0));
            }
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                x0[k] = ap0[k];
                x1[k] = ap1[k];
            }
            if constexpr (HOOK) prefetch();
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                acc = __builtin_amdgcn_mfma_f32_4x4x1f32(x0[k], y0[k], acc, 0, 0, 0);
                acc2 = __builtin_amdgcn_mfma_f32_4x4x1f32(x1[k], y1[k], acc2, 0, 0, 0);
            }
        };
        using R0 = std::integral_constant<int, 0>;
        using R1 = std::integral_constant<int, 1>;
        using NOH = std::integral_constant<bool, false>;
        using YH = std::integral_constant<bool, true>;
        const int G0 = (cnt0 + 1) >> 1, G = G0 + ((cnt1 + 1) >> 1);
        for (int g = 0; g < G - 1; ++g) {
            if (g < G0)
                grp(R0{}, NOH{}, 2 * g);
            else
                grp(R1{}, NOH{}, 2 * (g - G0));
        }
        if (G > 0) {
            if (G - 1 < G0)
                grp(R0{}, YH{}, 2 * (G - 1));
            else
                grp(R1{}, YH{}, 2 * (G - 1 - G0));
        } else {
            prefetch();
        }
        a0 += a0b;
        a1 += a1b;
        wave_sync_lds();  // the area takes the next column's lists
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            if (!C.val[i]) continue;
            const f32x4 &acc = i ? a1 : a0;
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                const uint32_t e = C.off[i] + v * 9;
                float o = (float)ep.alpha * acc[v];
                if (Prev) o = fmaf((float)ep.beta, C.prev[i][v], o);
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, o), r_out, (int)(e * 4), 0, 0);
                const double od = (double)o;
                if constexpr (MAXACC == 1)
                    if (ep.nacc > 0)
                        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, C.acc[i][v] + wq[0] * od), r_acc[0],
                                                              (int)(e * 8), 0, 0);
                if constexpr (MAXACC > 1) {
#pragma unroll
                    for (int qa = 0; qa < MAXACC; ++qa)
                        if (qa < ep.nacc) {
                            const double a = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r_acc[qa], (int)(e * 8), 0, 0));
                            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, a + wq[qa] * od), r_acc[qa],
                                                                  (int)(e * 8), 0, 0);
                        }
                }
                if (ep.hist) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, o), r_hist, (int)(e * 4), 0, 0);
                if (row0 + i == jc && 3 * (slot / 3) + v == bcol) tr += od;
            }
        }
    };
    if (nj > 0) {
        Set S0, S1;
        int jj = wave;
        lrec(jj, S0);
        lrow(S0);
        lrec(jj + NW, S1);
        for (; jj < nj; jj += 2 * NW) {
            column(S0, S1, jj);
            if (jj + NW >= nj) break;
            column(S1, S0, jj + NW);
        }
    }
    if (ep.trace_partial) {
        const double sm = bsum<NT>(tr);
        if (threadIdx.x == 0) ep.trace_partial[tile] = sm;
    }
}

template <int NW>
hipError_t launch_lean9(const ListedPlanDev &plan, const ProductOperands &ops, const Epilogue &ep,
                        hipStream_t st, size_t *lds_out) {
    const size_t lds = lean9_lds<NW>(plan).total;
    if (lds_out) {
        *lds_out = lds;
        return hipSuccess;
    }
    if (plan.ntiles == 0) return hipSuccess;
    if (plan.entry_width != 1 || plan.cmax != 2 || !plan.off31) return hipErrorInvalidValue;
    if (ep.nacc > 4) return hipErrorInvalidValue;
    static int raised_device = -1;
    static size_t raised_to = 0;
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (lds > 65536 && (raised_device != dev || raised_to < lds)) {
        hipError_t e = hipFuncSetAttribute((const void *)k_lean9<NW, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_lean9<NW, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_lean9<NW, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        raised_device = dev;
        raised_to = lds;
    }
    const int nt8 = (plan.ntiles + 7) & ~7;
    if (ep.nacc > 1)
        hipLaunchKernelGGL((k_lean9<NW, 4>), dim3(nt8), dim3(64 * NW), lds, st, plan, ops, ep);
    else if (ep.nacc == 1)
        hipLaunchKernelGGL((k_lean9<NW, 1>), dim3(nt8), dim3(64 * NW), lds, st, plan, ops, ep);
    else
        hipLaunchKernelGGL((k_lean9<NW, 0>), dim3(nt8), dim3(64 * NW), lds, st, plan, ops, ep);
    return hipGetLastError();
}

template <typename T, int B, int CMAX>
struct LVariant {
    // 1: float32 4x4x1 MFMA, 2: float64 4x4x4 MFMA, 0: vector ALU dot products
    static constexpr int MODE = (B == 4 && CMAX == 4) ? (std::is_same<T, float>::value ? 1 : 2) : 0;
    static constexpr int NW = sizeof(T) == 4 ? 8 : 4;
    // the last three ids of each MFMA mode are the output-stationary kernel
    // (kernels_stat.hip) on the plan's groups
    static constexpr int COUNT = MODE == 0 ? 1 : (MODE == 1 ? 27 : 13);
    // variants 4, 5 (pipelined hit groups), 10-15 (6- and 8-hit groups) and
    // 16-23 (free slot assignment) are float32 only
    static bool ok(int v) { return v >= 0 && v < COUNT && (MODE == 1 || (v != 4 && v != 5)); }
};

template <typename T, int B, int CMAX, int NW, int MODE, int EW, bool BD, bool PIPE, bool NTH,
          int G, bool SB, int MAXACC, bool PAD>
hipError_t launch_a(const ListedPlanDev &plan, const ProductOperands &ops, const Epilogue &ep,
                    hipStream_t st, size_t *lds_out);

// accumulator count is a template bound: chains with at most one float64
// sum (the common case) keep fewer registers
template <typename T, int B, int CMAX, int NW, int MODE, int EW, bool BD, bool PIPE = false,
          bool NTH = false, int G = 4, bool SB = false, bool PAD = false>
hipError_t launch_v(const ListedPlanDev &plan, const ProductOperands &ops, const Epilogue &ep,
                    hipStream_t st, size_t *lds_out) {
    if (ep.nacc <= 1) return launch_a<T, B, CMAX, NW, MODE, EW, BD, PIPE, NTH, G, SB, 1, PAD>(plan, ops, ep, st, lds_out);
    return launch_a<T, B, CMAX, NW, MODE, EW, BD, PIPE, NTH, G, SB, 4, PAD>(plan, ops, ep, st, lds_out);
}

template <typename T, int B, int CMAX, int NW, int MODE, int EW, bool BD, bool PIPE, bool NTH,
          int G, bool SB, int MAXACC, bool PAD>
hipError_t launch_a(const ListedPlanDev &plan, const ProductOperands &ops, const Epilogue &ep,
                    hipStream_t st, size_t *lds_out) {
    const size_t lds = listed_lds<T, B, NW, EW, BD>(plan).total;
    if (lds_out) {
        *lds_out = lds;
        return hipSuccess;
    }
    if (plan.ntiles == 0) return hipSuccess;
    const void *fn = (const void *)k_listed<T, B, CMAX, NW, MODE, EW, BD, PIPE, NTH, G, SB, MAXACC, PAD>;
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
    hipLaunchKernelGGL((k_listed<T, B, CMAX, NW, MODE, EW, BD, PIPE, NTH, G, SB, MAXACC, PAD>), dim3(nt8), dim3(64 * NW), lds, st,
                       plan, ops, ep);
    return hipGetLastError();
}

template <typename T, int B, int CMAX, int EW>
hipError_t launch_l(const ListedPlanDev &plan, const ProductOperands &ops, const Epilogue &ep,
                    hipStream_t st, size_t *lds_out) {
    typedef LVariant<T, B, CMAX> V;
    constexpr int NW = V::NW;
    constexpr int MODE = V::MODE;
    if constexpr (MODE == 0) {
        if (plan.variant == 0) return launch_v<T, B, CMAX, NW, MODE, EW, false>(plan, ops, ep, st, lds_out);
        if constexpr (std::is_same<T, float>::value && B == 9 && CMAX == 2) {
            // 9 x 9 blocks on the matrix cores; 3, 4: pipelined columns
            // (k_lean9) with 8 or 4 waves
            if (plan.variant == 3) return launch_lean9<8>(plan, ops, ep, st, lds_out);
            if (plan.variant == 4) return launch_lean9<4>(plan, ops, ep, st, lds_out);
            if (plan.variant == 1 || plan.variant == 2) {
                if (ep.nacc <= 1) {
                    if (plan.variant == 1) return launch_9<4, EW, 1>(plan, ops, ep, st, lds_out);
                    return launch_9<8, EW, 1>(plan, ops, ep, st, lds_out);
                }
                if (plan.variant == 1) return launch_9<4, EW, 4>(plan, ops, ep, st, lds_out);
                return launch_9<8, EW, 4>(plan, ops, ep, st, lds_out);
            }
        }
        return hipErrorInvalidValue;
    } else {
        {
            // the last three ids: the output-stationary kernel on the plan's groups
            const int v0 = MODE == 1 ? kStatVariantF32 : kStatVariantF64;
            const int d = plan.variant - v0;
            if (d >= 0) {
                if (d > 2) return hipErrorInvalidValue;
                const int nw = MODE == 1 ? (d == 0 ? 8 : d == 1 ? 4 : 16) : (d == 0 ? 4 : d == 1 ? 8 : 16);
                return launch_stat_product(MODE == 1 ? kStatF32 : kStatF64, nw, plan, ops, ep, st, lds_out);
            }
        }
        switch (plan.variant) {
            case 0: return launch_v<T, B, CMAX, NW, MODE, EW, false>(plan, ops, ep, st, lds_out);
            case 1: return launch_v<T, B, CMAX, NW, MODE, EW, true>(plan, ops, ep, st, lds_out);
            case 2: return launch_v<T, B, CMAX, 2 * NW, MODE, EW, true>(plan, ops, ep, st, lds_out);
            case 3: return launch_v<T, B, CMAX, NW / 2, MODE, EW, true>(plan, ops, ep, st, lds_out);
            case 4:
                if constexpr (MODE == 1) return launch_v<T, B, CMAX, NW, MODE, EW, true, true>(plan, ops, ep, st, lds_out);
                return hipErrorInvalidValue;
            case 5:
                if constexpr (MODE == 1) return launch_v<T, B, CMAX, 2 * NW, MODE, EW, true, true>(plan, ops, ep, st, lds_out);
                return hipErrorInvalidValue;
            case 6: return launch_v<T, B, CMAX, NW, MODE, EW, true, false, true>(plan, ops, ep, st, lds_out);
            case 7: return launch_v<T, B, CMAX, 2 * NW, MODE, EW, true, false, true>(plan, ops, ep, st, lds_out);
            case 8: return launch_v<T, B, CMAX, NW, MODE, EW, true, false, false, 4, true>(plan, ops, ep, st, lds_out);
            case 9: return launch_v<T, B, CMAX, 2 * NW, MODE, EW, true, false, false, 4, true>(plan, ops, ep, st, lds_out);
            case 10:
                if constexpr (MODE == 1) return launch_v<T, B, CMAX, NW, MODE, EW, true, false, false, 6, true>(plan, ops, ep, st, lds_out);
                return hipErrorInvalidValue;
            case 11:
                if constexpr (MODE == 1) return launch_v<T, B, CMAX, 2 * NW, MODE, EW, true, false, false, 6, true>(plan, ops, ep, st, lds_out);
                return hipErrorInvalidValue;
            case 12:
                if constexpr (MODE == 1) return launch_v<T, B, CMAX, NW, MODE, EW, true, false, false, 8, true>(plan, ops, ep, st, lds_out);
                return hipErrorInvalidValue;
            case 13:
                if constexpr (MODE == 1) return launch_v<T, B, CMAX, 2 * NW, MODE, EW, true, false, false, 8, true>(plan, ops, ep, st, lds_out);
                return hipErrorInvalidValue;
            case 14:
                if constexpr (MODE == 1) return launch_v<T, B, CMAX, NW, MODE, EW, true, false, false, 8, true, true>(plan, ops, ep, st, lds_out);
                return hipErrorInvalidValue;
            case 15:
                if constexpr (MODE == 1) return launch_v<T, B, CMAX, NW, MODE, EW, true, false, false, 6, true, true>(plan, ops, ep, st, lds_out);
                return hipErrorInvalidValue;
            case 16:
                if constexpr (MODE == 1 && EW == 1) return launch_lean<8, 8>(plan, ops, ep, st, lds_out);
                return hipErrorInvalidValue;
            case 17:
                if constexpr (MODE == 1 && EW == 1) return launch_lean<12, 8>(plan, ops, ep, st, lds_out);
                return hipErrorInvalidValue;
            case 18:
                if constexpr (MODE == 1 && EW == 1) return launch_lean<8, 4>(plan, ops, ep, st, lds_out);
                return hipErrorInvalidValue;
            case 19:
                if constexpr (MODE == 1 && EW == 1) return launch_lean<16, 4>(plan, ops, ep, st, lds_out);
                return hipErrorInvalidValue;
            case 20:
                if constexpr (MODE == 1 && EW == 1) return launch_lean<8, 8, true>(plan, ops, ep, st, lds_out);
                return hipErrorInvalidValue;
            case 21:
                if constexpr (MODE == 1 && EW == 1) return launch_lean<8, 4, true>(plan, ops, ep, st, lds_out);
                return hipErrorInvalidValue;
            case 22:
                if constexpr (MODE == 1 && EW == 1) return launch_lean<16, 4, true>(plan, ops, ep, st, lds_out);
                return hipErrorInvalidValue;
            case 23:
                if constexpr (MODE == 1 && EW == 1) return launch_lean<10, 4, true>(plan, ops, ep, st, lds_out);
                return hipErrorInvalidValue;
            default: return hipErrorInvalidValue;
        }
    }
}

template <typename T, int B, int CMAX>
hipError_t launch_lc(const ListedPlanDev &plan, const ProductOperands &ops, const Epilogue &ep,
                     hipStream_t st, size_t *lds_out) {
    if (plan.entry_width == 1) return launch_l<T, B, CMAX, 1>(plan, ops, ep, st, lds_out);
    if (plan.entry_width == 2) return launch_l<T, B, CMAX, 2>(plan, ops, ep, st, lds_out);
    return hipErrorInvalidValue;
}

template <typename T, int B>
hipError_t launch_lb(const ListedPlanDev &plan, const ProductOperands &ops, const Epilogue &ep,
                     hipStream_t st, size_t *lds_out) {
    switch (plan.cmax) {
        case 1: return launch_lc<T, B, 1>(plan, ops, ep, st, lds_out);
        case 2: return launch_lc<T, B, 2>(plan, ops, ep, st, lds_out);
        case 4: return launch_lc<T, B, 4>(plan, ops, ep, st, lds_out);
        default: return hipErrorInvalidValue;
    }
}

hipError_t dispatch_listed(int dtype, int b, const ListedPlanDev &plan, const ProductOperands &ops,
                           const Epilogue &ep, hipStream_t st, size_t *lds_out) {
    if (ops.opmode != 0) {
        // bfloat16 operands: the output-stationary kernel on float32 storage
        const int d = plan.variant - kStatVariantF32;
        if (dtype != 1 || b != 4 || d < 0 || d > 2) return hipErrorInvalidValue;
        return launch_stat_product(ops.opmode, d == 0 ? 8 : d == 1 ? 4 : 16, plan, ops, ep, st, lds_out);
    }
    if (b == 4) {
        // the output-stationary ids, for tiles of any height
        const int d = plan.variant - (dtype == 1 ? kStatVariantF32 : kStatVariantF64);
        if (d >= 0 && d <= 2) {
            const int nw = dtype == 1 ? (d == 0 ? 8 : d == 1 ? 4 : 16) : (d == 0 ? 4 : d == 1 ? 8 : 16);
            return launch_stat_product(dtype == 1 ? kStatF32 : kStatF64, nw, plan, ops, ep, st, lds_out);
        }
    }
    if (dtype == 0 && b == 4) return launch_lb<double, 4>(plan, ops, ep, st, lds_out);
    if (dtype == 0 && b == 9) return launch_lb<double, 9>(plan, ops, ep, st, lds_out);
    if (dtype == 1 && b == 4) return launch_lb<float, 4>(plan, ops, ep, st, lds_out);
    if (dtype == 1 && b == 9) return launch_lb<float, 9>(plan, ops, ep, st, lds_out);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_listed_product(int dtype, int b, const ListedPlanDev &plan,
                                 const ProductOperands &ops, const Epilogue &ep, hipStream_t st) {
    return dispatch_listed(dtype, b, plan, ops, ep, st, nullptr);
}

int listed_product_variants(int dtype, int b, const ListedPlanDev &plan) {
    if (b == 9 && dtype == 1 && plan.cmax == 2) return 5;  // VALU, MFMA with 4 or 8 waves, pipelined MFMA
    if (b != 4) return 1;
    // b = 4: every id (other tile heights than 4 take the output-stationary ones)
    return dtype == 0 ? LVariant<double, 4, 4>::COUNT : LVariant<float, 4, 4>::COUNT;
}

bool listed_product_variant_ok(int dtype, int b, const ListedPlanDev &plan, int v, int opmode) {
    const bool stat_ok = b == 4 && plan.st_goff && plan.st_g == (dtype == 0 ? 4 : 16);
    if (opmode != 0) return dtype == 1 && stat_ok && v >= kStatVariantF32 && v <= kStatVariantF32 + 2;
    if (b == 9 && dtype == 1 && plan.cmax == 2)
        return v >= 0 && v < 5 && (v < 3 || (plan.off31 && plan.entry_width == 1));
    const int v0 = dtype == 0 ? kStatVariantF64 : kStatVariantF32;
    // b = 4 tiles of other heights (chosen by the tile tuner): the
    // output-stationary kernel only, which takes any tile of 1..4 rows
    if (b == 4 && plan.cmax != 4) return stat_ok && v >= v0 && v <= v0 + 2;
    if (b != 4 || plan.cmax != 4) return v == 0;
    if (v >= v0) return v <= v0 + 2 && stat_ok;
    if (v >= 16 && !(dtype == 1 && plan.lean_rec && plan.entry_width == 1)) return false;
    return dtype == 0 ? LVariant<double, 4, 4>::ok(v) : LVariant<float, 4, 4>::ok(v);
}

size_t listed_product_lds_bytes(int dtype, int b, const ListedPlanDev &plan, int opmode) {
    size_t lds = 0;
    ProductOperands ops{};
    ops.opmode = opmode;
    if (dispatch_listed(dtype, b, plan, ops, Epilogue{}, nullptr, &lds) != hipSuccess)
        return (size_t)-1;
    return lds;
}

}  // namespace chess
