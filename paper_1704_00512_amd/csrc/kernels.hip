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

template <typename T, int B, int CMAX>
__global__ __launch_bounds__(kWG) void k_masked_product(ProductPlanDev plan, ProductOperands ops,
                                                        Epilogue ep) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    constexpr int BB = B * B;
    constexpr int NEL = CMAX * BB;
    constexpr int NE = (NEL + 63) / 64;

    const int ntiles = plan.ntiles;
    const int nt8 = (ntiles + 7) & ~7;
    const int w = blockIdx.x;
    // XCD-aware mapping: workgroup w runs on XCD w % 8; give each XCD a
    // contiguous range of tiles.
    const int tile = (w & 7) * (nt8 >> 3) + (w >> 3);
    if (tile >= ntiles) return;

    const int row0 = plan.tile_row0[tile];
    const int c = plan.tile_row0[tile + 1] - row0;
    const int64_t ab0 = ops.a_rp[row0];
    const int nab = (int)(ops.a_rp[row0 + c] - ab0);
    const int hcap = 1 << plan.hcap_log2;
    const unsigned hmask = (unsigned)hcap - 1u;

    T *As = reinterpret_cast<T *>(smem);
    int *hkey = reinterpret_cast<int *>(smem + (size_t)plan.lds_ablocks * BB * sizeof(T));
    short *hval = reinterpret_cast<short *>(hkey + hcap);
    unsigned short *upos = reinterpret_cast<unsigned short *>(hval + hcap);

    // stage this tile's rows of A (contiguous in block CSR)
    {
        const T *Ag = reinterpret_cast<const T *>(ops.a_val) + ab0 * BB;
        const int n = nab * BB;
        for (int x = threadIdx.x; x < n; x += kWG) As[x] = Ag[x];
        for (int x = threadIdx.x; x < hcap; x += kWG) hkey[x] = -1;
    }
    __syncthreads();
    const int64_t u0 = plan.u_off[tile];
    const int nu = (int)(plan.u_off[tile + 1] - u0);
    for (int k = threadIdx.x; k < nu; k += kWG) {
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

    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;

    int ei[NE], er[NE], es[NE];
    int64_t cbase[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int e = lane + 64 * q;
        ei[q] = e / BB;
        er[q] = (e % BB) / B;
        es[q] = e % B;
        cbase[q] = (ei[q] < c) ? ops.c_rp[row0 + ei[q]] : -1;
    }

    const int64_t j0 = plan.j_off[tile];
    const int nj = (int)(plan.j_off[tile + 1] - j0);
    const T *Bt = reinterpret_cast<const T *>(ops.bt_val);
    T *Cout = reinterpret_cast<T *>(ops.c_out);
    const T *Prev = reinterpret_cast<const T *>(ep.prev);
    T *Hist = reinterpret_cast<T *>(ep.hist);
    const T alpha = (T)ep.alpha;
    const T beta = (T)ep.beta;
    double tr = 0.0;

    for (int jj = wave; jj < nj; jj += kWG / 64) {
        const int j = plan.j_cols[j0 + jj];
        int64_t outp[NE];
        T acc[NE];
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            acc[q] = (T)0;
            outp[q] = -1;
            if (ei[q] < c) {
                const unsigned short op = plan.j_pos[(j0 + jj) * CMAX + ei[q]];
                if (op != 0xFFFF) outp[q] = cbase[q] + op;
            }
        }
        const int64_t s0 = ops.bt_rp[j];
        const int64_t s1 = ops.bt_rp[j + 1];
        for (int64_t sl = s0; sl < s1; ++sl) {
            const int l = ops.bt_ci[sl];
            unsigned h = hash_slot(l, plan.hcap_log2);
            int k = -1;
            while (true) {
                const int key = hkey[h];
                if (key == l) {
                    k = hval[h];
                    break;
                }
                if (key < 0) break;
                h = (h + 1u) & hmask;
            }
            if (k < 0) continue;
            const T *bb = Bt + sl * BB;
#pragma unroll
            for (int q = 0; q < NE; ++q) {
                if (outp[q] >= 0) {
                    const unsigned short pa = upos[k * CMAX + ei[q]];
                    if (pa != 0xFFFF) {
                        const T *a = As + (int)pa * BB + er[q] * B;
                        const T *bs = bb + es[q] * B;
                        T s = (T)0;
#pragma unroll
                        for (int t = 0; t < B; ++t) s = fma(a[t], bs[t], s);
                        acc[q] += s;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            if (outp[q] >= 0) {
                const int64_t off = outp[q] * BB + er[q] * B + es[q];
                T o = alpha * acc[q];
                if (Prev) o = fma(beta, Prev[off], o);
                Cout[off] = o;
                const double od = (double)o;
                for (int qa = 0; qa < ep.nacc; ++qa) ep.acc[qa][off] += ep.coef[qa] * od;
                if (Hist) Hist[off] = o;
                if (row0 + ei[q] == j && er[q] == es[q]) tr += od;
            }
        }
    }
    if (ep.trace_partial) {
        const double s = block_sum(tr);
        if (threadIdx.x == 0) ep.trace_partial[tile] = s;
    }
}

template <typename T, int B, int CMAX>
size_t product_lds(const ProductPlanDev &plan) {
    const size_t hcap = (size_t)1 << plan.hcap_log2;
    size_t bytes = (size_t)plan.lds_ablocks * B * B * sizeof(T) + hcap * 4 + hcap * 2 +
                   (size_t)plan.max_u * CMAX * 2;
    return (bytes + 15) & ~(size_t)15;
}

template <typename T, int B, int CMAX>
hipError_t launch_product_t(const ProductPlanDev &plan, const ProductOperands &ops,
                            const Epilogue &ep, hipStream_t st) {
    if (plan.ntiles == 0) return hipSuccess;
    const size_t lds = product_lds<T, B, CMAX>(plan);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)k_masked_product<T, B, CMAX>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int nt8 = (plan.ntiles + 7) & ~7;
    hipLaunchKernelGGL((k_masked_product<T, B, CMAX>), dim3(nt8), dim3(kWG), lds, st, plan, ops,
                       ep);
    return hipGetLastError();
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
