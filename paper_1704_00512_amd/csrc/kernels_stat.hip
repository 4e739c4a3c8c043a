// The Chebyshev-step product with output-stationary MFMA slots (b = 4).
//
// The step computes Y = P_C o (A Bt^T) on a fixed pattern (Eq. 4 truncated as
// in Sec. "Truncation to a fixed sparsity pattern"): output block (i, j) sums
// A[i, l] Bt[j, l]^T over the l shared by row i of A and row j of Bt.  The
// plan (built once per pattern triple on the host) lists, for every output
// block, its hits as (position of l in A row i, position of l in Bt row j).
//
// Work decomposition: one workgroup per tile of <= 4 consecutive rows of A,
// whose blocks are copied to LDS once, each row followed by one block of
// zeros.  The tile's output blocks, sorted by hit count, form groups of G (16
// for the single-precision operand modes, 4 for float64).  A wave takes a
// group; each MFMA slot owns one output block of it for all R rounds of the
// group (R = the group's largest hit count, rounded up to 8), taking one hit
// per round; lists shorter than R are padded with the row's zero block, so
// the padded products are exact zeros and the loop has no conditions.  There
// is no reduction across slots: after the rounds each slot holds its finished
// block, which the fused epilogue stores directly.
//
// Operand modes (the A tile in LDS, Bt rows from global memory through a
// buffer descriptor):
//   kF32:    float32 operands, v_mfma_f32_4x4x1_16b_f32 (16 slots; four MFMAs
//            of one k each form a 4x4x4 block product);
//   kBF16:   bfloat16 operands (round to nearest even), float32 accumulation,
//            v_mfma_f32_4x4x4_16b_bf16 (one MFMA per block product);
//   kBF16X3: each float32 operand split as hi + lo with hi = bf16(x),
//            lo = bf16(x - hi); the product is hi*hi + hi*lo + lo*hi (three
//            bf16 MFMAs, lo*lo dropped), float32 accumulation;
//   kF64:    float64, v_mfma_f64_4x4x4_4b_f64 (4 slots of 16 lanes, one MFMA
//            per block product).
// The chain's T_k are stored in float32 for the first three modes and in
// float64 for the last; the epilogue is that of kernels.h (Epilogue).
//
// MFMA lane layouts (16-slot forms): lane 4 s + q of slot s supplies row q of
// the Bt block as the first operand and row q of the A block as the second;
// the result lane 4 s + q, register v, is C[v][q] = sum_k Bt[v][k] A[q][k] =
// Y[q][v]: each lane ends with row q of its slot's output block, 16
// contiguous bytes.  float64: operand lane 16 t + 4 s + x holds A[x][t] and
// Bt[x][t]; result lane 16 r + 4 s + c holds Y[r][c].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "kernels.h"

namespace chess {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

template <int MODE>
struct StatMode {
    static constexpr int G = MODE == kStatF64 ? 4 : 16;  // slots (output blocks) per group
    // LDS bytes per A block: float32 / hi+lo pair 64, bf16 32, float64 128
    static constexpr int AB = MODE == kStatF64 ? 128 : (MODE == kStatBF16 ? 32 : 64);
    // bytes per Bt block in each operand array
    static constexpr int BB = MODE == kStatF64 ? 128 : (MODE == kStatF32 ? 64 : 32);
    // bytes per stored block of A (the chain's storage precision)
    static constexpr int SB = MODE == kStatF64 ? 128 : 64;
};

__device__ inline __amdgpu_buffer_rsrc_t mkrsrc(const void *p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, 0x7FFFFFFF, 0x00020000);
}

// bfloat16 bits of x, rounded to nearest even
__device__ inline unsigned int bf16_bits(float x) {
    const __bf16 h = (__bf16)x;
    return (unsigned int)__builtin_bit_cast(unsigned short, h);
}
__device__ inline float bf16_value(unsigned int bits) { return __builtin_bit_cast(float, bits << 16); }

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int NT>
__device__ inline double block_sum(double v) {
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

template <int MODE, int NW, int MAXACC>
__global__ __launch_bounds__(64 * NW) void k_stat(ListedPlanDev plan, ProductOperands ops, Epilogue ep) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    typedef StatMode<MODE> SM;
    constexpr int G = SM::G, AB = SM::AB, BB = SM::BB, SB = SM::SB;
    constexpr int NT = 64 * NW;
    constexpr int NACC = MAXACC > 0 ? MAXACC : 1;
    const int ntiles = plan.ntiles;
    const int nt8 = (ntiles + 7) & ~7;
    const int wg = blockIdx.x;
    // XCD-aware: workgroup w runs on XCD w mod 8; each XCD gets a contiguous
    // range of tiles (neighbouring atoms share that XCD's L2 for Bt rows)
    const int tile = (wg & 7) * (nt8 >> 3) + (wg >> 3);
    if (tile >= ntiles) return;
    const int row0 = plan.tile_row0[tile];
    if (tile_finished(ep, tile, row0)) return;
    const int c = plan.tile_row0[tile + 1] - row0;
    const int64_t ab0 = ops.a_rp[row0];
    // cumulative row ends in source blocks (rows past c have length 0)
    const int e0 = (int)(ops.a_rp[row0 + 1] - ab0);
    const int e1 = (1 < c) ? (int)(ops.a_rp[row0 + 2] - ab0) : e0;
    const int e2 = (2 < c) ? (int)(ops.a_rp[row0 + 3] - ab0) : e1;
    const int e3 = (3 < c) ? (int)(ops.a_rp[row0 + 4] - ab0) : e2;
    {
        // A tile -> LDS: source block x of tile row r goes to block x + r
        // (one zero block after each earlier row), converted to the operand
        // form; 16-byte chunks of the stored blocks
        constexpr int CPB = SB / 16;
        const u32x4 *src = reinterpret_cast<const u32x4 *>(reinterpret_cast<const unsigned char *>(ops.a_val) +
                                                           ab0 * SB);
        const int nchunk = e3 * CPB;
        for (int x = threadIdx.x; x < nchunk; x += NT) {
            const int blk = x / CPB, part = x % CPB;
            const int r = (blk >= e0) + (blk >= e1) + (blk >= e2);
            const int dblk = blk + r;
            const u32x4 v = src[x];
            if constexpr (MODE == kStatF32 || MODE == kStatF64) {
                *reinterpret_cast<u32x4 *>(smem + (size_t)dblk * AB + part * 16) = v;
            } else {
                const f32x4 f = __builtin_bit_cast(f32x4, v);
                unsigned int h[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) h[k] = bf16_bits(f[k]);
                u32x2 hp = {h[0] | (h[1] << 16), h[2] | (h[3] << 16)};
                *reinterpret_cast<u32x2 *>(smem + (size_t)dblk * AB + part * 8) = hp;
                if constexpr (MODE == kStatBF16X3) {
                    unsigned int l[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) l[k] = bf16_bits(f[k] - bf16_value(h[k]));
                    u32x2 lp = {l[0] | (l[1] << 16), l[2] | (l[3] << 16)};
                    *reinterpret_cast<u32x2 *>(smem + (size_t)dblk * AB + 32 + part * 8) = lp;
                }
            }
        }
        // the zero block of row r sits at block e_r + r
        constexpr int ZC = AB / 16;
        for (int x = threadIdx.x; x < c * ZC; x += NT) {
            const int r = x / ZC, part = x % ZC;
            const int er = r == 0 ? e0 : r == 1 ? e1 : r == 2 ? e2 : e3;
            *reinterpret_cast<u32x4 *>(smem + (size_t)(er + r) * AB + part * 16) = u32x4{0u, 0u, 0u, 0u};
        }
    }
    __syncthreads();

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    int slot, ao;
    if constexpr (MODE == kStatF64) {
        slot = (lane >> 2) & 3;
        ao = ((lane & 3) * 4 + (lane >> 4)) * 8;
    } else {
        slot = lane >> 2;
        ao = (MODE == kStatF32) ? (lane & 3) * 16 : (lane & 3) * 8;
    }
    const int bo = ao & (BB - 1);
    double wq[NACC];
    {
        const int sys = ep.row_sys ? ep.row_sys[row0] : 0;
#pragma unroll
        for (int qa = 0; qa < NACC; ++qa)
            wq[qa] = (qa < MAXACC && ep.row_sys && ep.coef_sys[qa]) ? ep.coef_sys[qa][sys] : ep.coef[qa];
    }
    const __amdgpu_buffer_rsrc_t r_list = mkrsrc(plan.st_list);
    const __amdgpu_buffer_rsrc_t r_bt = mkrsrc(MODE == kStatF32 || MODE == kStatF64 ? ops.bt_val : ops.bt_hi);
    const __amdgpu_buffer_rsrc_t r_btlo = mkrsrc(MODE == kStatBF16X3 ? ops.bt_lo : ops.bt_val);
    const __amdgpu_buffer_rsrc_t r_prev = mkrsrc(ep.prev ? ep.prev : ops.a_val);
    const __amdgpu_buffer_rsrc_t r_out = mkrsrc(ops.c_out);
    const __amdgpu_buffer_rsrc_t r_hist = mkrsrc(ep.hist ? ep.hist : ops.c_out);
    const __amdgpu_buffer_rsrc_t r_a = mkrsrc(ops.a_val);  // T_m in storage precision
    const bool dots = ep.sq_partial != nullptr;
    __amdgpu_buffer_rsrc_t r_acc[NACC];
#pragma unroll
    for (int qa = 0; qa < NACC; ++qa) r_acc[qa] = mkrsrc((qa < ep.nacc) ? ep.acc[qa] : ep.acc[0]);
    typedef __attribute__((address_space(3))) const unsigned char lds_u8;
    lds_u8 *As = (lds_u8 *)smem;
    double tr = 0.0, dsq = 0.0, dxy = 0.0;
    const int g0 = plan.st_goff[tile], g1 = plan.st_goff[tile + 1];
    for (int g = g0 + wave; g < g1; g += NW) {
        const int li = plan.st_ginfo[2 * g];
        const int rw = plan.st_ginfo[2 * g + 1];
        const int nch = (rw & 0xFFFF) >> 3;
        const unsigned int dmask = (unsigned int)rw >> 16;
        const u32x2 sr = *reinterpret_cast<const u32x2 *>(plan.st_slot + 2 * ((size_t)g * G + slot));
        const uint32_t outb = sr.x;
        const bool valid = outb != 0xFFFFFFFFu;
        const uint32_t bbase = (sr.y & 0x3FFFFFu) * BB + bo;
        lds_u8 *abase = As + (sr.y >> 22) * AB + ao;
        const uint32_t lbase = (uint32_t)(li + slot * nch) * 16u;
        // epilogue operands of this lane, loaded while the rounds run; lanes
        // without an output read element 0 and drop the values
        uint32_t eoff;
        if constexpr (MODE == kStatF64)
            eoff = valid ? outb * 16u + (lane >> 4) * 4 + (lane & 3) : 0u;
        else
            eoff = valid ? outb * 16u + (lane & 3) * 4 : 0u;
        typedef typename std::conditional<MODE == kStatF64, double, f32x4>::type OutT;
        OutT prev;
        double accv[NACC][MODE == kStatF64 ? 1 : 4];
        if constexpr (MODE == kStatF64) {
            prev = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r_prev, (int)(eoff * 8), 0, 0));
#pragma unroll
            for (int qa = 0; qa < MAXACC; ++qa)
                accv[qa][0] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r_acc[qa], (int)(eoff * 8), 0, 0));
        } else {
            prev = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r_prev, (int)(eoff * 4), 0, 0));
#pragma unroll
            for (int qa = 0; qa < MAXACC; ++qa) {
                const f64x2 lo2 = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r_acc[qa], (int)(eoff * 8), 0, 0));
                const f64x2 hi2 = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r_acc[qa], (int)(eoff * 8 + 16), 0, 0));
                accv[qa][0] = lo2[0];
                accv[qa][1] = lo2[1];
                accv[qa][2] = hi2[0];
                accv[qa][3] = hi2[1];
            }
        }
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        double dacc = 0.0;
        // hit lists: 8 rounds (8 two-byte entries) per 16-byte chunk, the
        // next two chunks prefetched (clamped to the last one)
        u32x4 ec = __builtin_amdgcn_raw_buffer_load_b128(r_list, (int)lbase, 0, 0);
        u32x4 en = __builtin_amdgcn_raw_buffer_load_b128(r_list, (int)(lbase + (nch > 1 ? 16 : 0)), 0, 0);
        for (int ch = 0; ch < nch; ++ch) {
            const u32x4 e = ec;
            ec = en;
            en = __builtin_amdgcn_raw_buffer_load_b128(r_list, (int)(lbase + 16 * min(ch + 2, nch - 1)), 0, 0);
            uint32_t apos[8], bpos[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t w2 = e[u >> 1] >> ((u & 1) * 16);
                apos[u] = w2 & 0xFFu;
                bpos[u] = (w2 >> 8) & 0xFFu;
            }
            if constexpr (MODE == kStatF32) {
                u32x4 bv[8];
                f32x4 av[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    bv[u] = __builtin_amdgcn_raw_buffer_load_b128(r_bt, (int)(bbase + bpos[u] * BB), 0, 0);
#pragma unroll
                for (int u = 0; u < 8; ++u) av[u] = *(const __attribute__((address_space(3))) f32x4 *)(abase + apos[u] * AB);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const f32x4 b = __builtin_bit_cast(f32x4, bv[u]);
                    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(b[0], av[u][0], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(b[1], av[u][1], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(b[2], av[u][2], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(b[3], av[u][3], acc, 0, 0, 0);
                }
            } else if constexpr (MODE == kStatBF16) {
                u32x2 bv[8], av[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    bv[u] = __builtin_amdgcn_raw_buffer_load_b64(r_bt, (int)(bbase + bpos[u] * BB), 0, 0);
#pragma unroll
                for (int u = 0; u < 8; ++u) av[u] = *(const __attribute__((address_space(3))) u32x2 *)(abase + apos[u] * AB);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    acc = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(__builtin_bit_cast(s16x4, bv[u]),
                                                                 __builtin_bit_cast(s16x4, av[u]), acc, 0, 0, 0);
            } else if constexpr (MODE == kStatBF16X3) {
                u32x2 bh[8], bl[8], ah[8], al[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    bh[u] = __builtin_amdgcn_raw_buffer_load_b64(r_bt, (int)(bbase + bpos[u] * BB), 0, 0);
                    bl[u] = __builtin_amdgcn_raw_buffer_load_b64(r_btlo, (int)(bbase + bpos[u] * BB), 0, 0);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    ah[u] = *(const __attribute__((address_space(3))) u32x2 *)(abase + apos[u] * AB);
                    al[u] = *(const __attribute__((address_space(3))) u32x2 *)(abase + apos[u] * AB + 32);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const s16x4 Bh = __builtin_bit_cast(s16x4, bh[u]), Bl = __builtin_bit_cast(s16x4, bl[u]);
                    const s16x4 Ah = __builtin_bit_cast(s16x4, ah[u]), Al = __builtin_bit_cast(s16x4, al[u]);
                    acc = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(Bl, Ah, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(Bh, Al, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(Bh, Ah, acc, 0, 0, 0);
                }
            } else {
                double bv[8], av[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    bv[u] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r_bt, (int)(bbase + bpos[u] * BB), 0, 0));
#pragma unroll
                for (int u = 0; u < 8; ++u) av[u] = *(const __attribute__((address_space(3))) double *)(abase + apos[u] * AB);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < 8; ++u) dacc = __builtin_amdgcn_mfma_f64_4x4x4f64(av[u], bv[u], dacc, 0, 0, 0);
            }
        }
        // fused epilogue
        if (valid) {
            if constexpr (MODE == kStatF64) {
                double o = ep.alpha * dacc;
                if (ep.prev) o = fma(ep.beta, prev, o);
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, o), r_out, (int)(eoff * 8), 0, 0);
#pragma unroll
                for (int qa = 0; qa < MAXACC; ++qa)
                    if (qa < ep.nacc)
                        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, fma(wq[qa], o, accv[qa][0])),
                                                              r_acc[qa], (int)(eoff * 8), 0, 0);
                if (ep.hist) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, o), r_hist, (int)(eoff * 8), 0, 0);
                if (((dmask >> slot) & 1u) && (lane >> 4) == (lane & 3)) tr += o;
                if (dots) {
                    const double a = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r_a, (int)(eoff * 8), 0, 0));
                    dsq += o * o;
                    dxy += o * a;
                }
            } else {
                f32x4 o;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    o[v] = (float)ep.alpha * acc[v];
                    if (ep.prev) o[v] = fmaf((float)ep.beta, prev[v], o[v]);
                }
                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, o), r_out, (int)(eoff * 4), 0, 0);
#pragma unroll
                for (int qa = 0; qa < MAXACC; ++qa) {
                    if (qa < ep.nacc) {
                        f64x2 lo2, hi2;
                        lo2[0] = fma(wq[qa], (double)o[0], accv[qa][0]);
                        lo2[1] = fma(wq[qa], (double)o[1], accv[qa][1]);
                        hi2[0] = fma(wq[qa], (double)o[2], accv[qa][2]);
                        hi2[1] = fma(wq[qa], (double)o[3], accv[qa][3]);
                        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, lo2), r_acc[qa], (int)(eoff * 8), 0, 0);
                        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, hi2), r_acc[qa], (int)(eoff * 8 + 16), 0, 0);
                    }
                }
                if (ep.hist) __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, o), r_hist, (int)(eoff * 4), 0, 0);
                if (dots) {
                    const f32x4 a = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r_a, (int)(eoff * 4), 0, 0));
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        dsq += (double)o[v] * o[v];
                        dxy += (double)o[v] * a[v];
                    }
                }
                if ((dmask >> slot) & 1u) {
                    const int q = lane & 3;
                    const float d = q == 0 ? o[0] : q == 1 ? o[1] : q == 2 ? o[2] : o[3];
                    tr += (double)d;
                }
            }
        }
    }
    if (ep.trace_partial) {
        const double s = block_sum<NT>(tr);
        if (threadIdx.x == 0) ep.trace_partial[tile] = s;
    }
    if (dots) {
        const double s1 = block_sum<NT>(dsq);
        const double s2 = block_sum<NT>(dxy);
        if (threadIdx.x == 0) {
            ep.sq_partial[tile] = s1;
            ep.xy_partial[tile] = s2;
        }
    }
}

template <int MODE, int NW, int MAXACC>
hipError_t launch_stat_a(const ListedPlanDev &plan, const ProductOperands &ops, const Epilogue &ep,
                         hipStream_t st, size_t *lds_out) {
    const size_t lds = (size_t)plan.st_ablocks * StatMode<MODE>::AB;
    if (lds_out) {
        *lds_out = lds;
        return hipSuccess;
    }
    if (plan.ntiles == 0) return hipSuccess;
    if (!plan.st_goff || plan.st_g != StatMode<MODE>::G) return hipErrorInvalidValue;
    const void *fn = (const void *)k_stat<MODE, NW, MAXACC>;
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
    hipLaunchKernelGGL((k_stat<MODE, NW, MAXACC>), dim3(nt8), dim3(64 * NW), lds, st, plan, ops, ep);
    return hipGetLastError();
}

template <int MODE, int NW>
hipError_t launch_stat_w(const ListedPlanDev &plan, const ProductOperands &ops, const Epilogue &ep,
                         hipStream_t st, size_t *lds_out) {
    if (ep.nacc <= 0) return launch_stat_a<MODE, NW, 0>(plan, ops, ep, st, lds_out);
    if (ep.nacc == 1) return launch_stat_a<MODE, NW, 1>(plan, ops, ep, st, lds_out);
    return launch_stat_a<MODE, NW, 4>(plan, ops, ep, st, lds_out);
}

template <int MODE>
hipError_t launch_stat_m(int nw, const ListedPlanDev &plan, const ProductOperands &ops, const Epilogue &ep,
                         hipStream_t st, size_t *lds_out) {
    switch (nw) {
        case 4: return launch_stat_w<MODE, 4>(plan, ops, ep, st, lds_out);
        case 8: return launch_stat_w<MODE, 8>(plan, ops, ep, st, lds_out);
        case 16: return launch_stat_w<MODE, 16>(plan, ops, ep, st, lds_out);
        default: return hipErrorInvalidValue;
    }
}

// bf16 hi (and lo) of n float32 values
__global__ void k_split_bf16(int64_t n, const float *in, unsigned short *hi, unsigned short *lo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = in[i];
    const unsigned int h = bf16_bits(x);
    hi[i] = (unsigned short)h;
    if (lo) lo[i] = (unsigned short)bf16_bits(x - bf16_value(h));
}

}  // namespace

hipError_t launch_stat_product(int mode, int nw, const ListedPlanDev &plan, const ProductOperands &ops,
                               const Epilogue &ep, hipStream_t st, size_t *lds_out) {
    switch (mode) {
        case kStatF32: return launch_stat_m<kStatF32>(nw, plan, ops, ep, st, lds_out);
        case kStatBF16: return launch_stat_m<kStatBF16>(nw, plan, ops, ep, st, lds_out);
        case kStatBF16X3: return launch_stat_m<kStatBF16X3>(nw, plan, ops, ep, st, lds_out);
        case kStatF64: return launch_stat_m<kStatF64>(nw, plan, ops, ep, st, lds_out);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_split_bf16(int64_t n, const float *in, unsigned short *hi, unsigned short *lo, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st, n, in, hi, lo);
    return hipGetLastError();
}

}  // namespace chess
