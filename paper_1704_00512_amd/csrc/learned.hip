// Kernels of the learned predictor of spectral bounds and mu: the matrix
// statistics it reads (row features of H') and the two-layer perceptron
// (forward pass, loss gradient, Adam update).
//
// Network: h = tanh(W1 x + b1), y = W2 h + b2 with x of 64 features, 128
// hidden units and 3 outputs; parameters flat and row-major:
// W1 [128][64], b1 [128], W2 [3][128], b2 [3].  Loss over a batch of B rows:
// L = 1 / (2 B) sum (y - t)^2.  The optional normalisation block
// `norm` = {x_mean[64], x_inv_std[64], y_mean[3], y_std[3]} maps raw
// features in and normalised outputs back.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/chess.h"
#include "kernels.h"

namespace chess {
namespace {

constexpr int NI = kMlpIn, NH = kMlpHidden, NO = kMlpOut;
static_assert(NH % 64 == 0, "hidden layer: whole waves");

// One workgroup of NH threads per batch row; thread h owns hidden unit h.
__global__ __launch_bounds__(NH) void k_mlp_forward(const float *__restrict__ p,
                                                    const float *__restrict__ norm,
                                                    const float *__restrict__ x, int batch,
                                                    float *__restrict__ hid,
                                                    float *__restrict__ y) {
    __shared__ float xs[NI];
    __shared__ float red[NO][NH / 64];
    const int row = blockIdx.x;
    const int h = threadIdx.x;
    if (row >= batch) return;
    for (int i = h; i < NI; i += NH) {
        float v = x[(size_t)row * NI + i];
        if (norm) v = (v - norm[i]) * norm[NI + i];
        xs[i] = v;
    }
    __syncthreads();
    const float *W1 = p;
    const float *b1 = W1 + NH * NI;
    const float *W2 = b1 + NH;
    const float *b2 = W2 + NO * NH;
    float a = b1[h];
#pragma unroll 8
    for (int i = 0; i < NI; ++i) a = fmaf(W1[h * NI + i], xs[i], a);
    const float t = tanhf(a);
    if (hid) hid[(size_t)row * NH + h] = t;
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        float v = W2[o * NH + h] * t;
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((h & 63) == 0) red[o][h >> 6] = v;
    }
    __syncthreads();
    if (h < NO) {
        float v = b2[h];
        for (int w = 0; w < NH / 64; ++w) v += red[h][w];
        if (norm) v = fmaf(v, norm[2 * NI + NO + h], norm[2 * NI + h]);
        y[(size_t)row * NO + h] = v;
    }
}

// dY = (y - t) / B and dH = (dY W2) o (1 - h^2); one thread per (row, unit).
__global__ void k_mlp_delta(const float *__restrict__ p, const float *__restrict__ hid,
                            const float *__restrict__ y, const float *__restrict__ t, int batch,
                            float *__restrict__ dy, float *__restrict__ dh) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)batch * NH) return;
    const int row = (int)(idx / NH), h = (int)(idx % NH);
    const float *W2 = p + NH * NI + NH;
    const float inv_b = 1.0f / (float)batch;
    float s = 0.0f;
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        const float d = (y[(size_t)row * NO + o] - t[(size_t)row * NO + o]) * inv_b;
        s = fmaf(d, W2[o * NH + h], s);
        if (h == 0) dy[(size_t)row * NO + o] = d;
    }
    const float hh = hid[(size_t)row * NH + h];
    dh[(size_t)row * NH + h] = s * (1.0f - hh * hh);
}

// Gradient: one thread per parameter, float64 sum over the rows in order.
__global__ void k_mlp_grad(const float *__restrict__ x, const float *__restrict__ hid,
                           const float *__restrict__ dy, const float *__restrict__ dh, int batch,
                           float *__restrict__ g) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (k < NH * NI) {
        const int h = k / NI, i = k % NI;
        for (int r = 0; r < batch; ++r) s += (double)dh[(size_t)r * NH + h] * x[(size_t)r * NI + i];
    } else if (k < NH * NI + NH) {
        const int h = k - NH * NI;
        for (int r = 0; r < batch; ++r) s += dh[(size_t)r * NH + h];
    } else if (k < NH * NI + NH + NO * NH) {
        const int q = k - NH * NI - NH, o = q / NH, h = q % NH;
        for (int r = 0; r < batch; ++r) s += (double)dy[(size_t)r * NO + o] * hid[(size_t)r * NH + h];
    } else if (k < kMlpParams) {
        const int o = k - NH * NI - NH - NO * NH;
        for (int r = 0; r < batch; ++r) s += dy[(size_t)r * NO + o];
    } else {
        return;
    }
    g[k] = (float)s;
}

// L = 1 / (2 B) sum (y - t)^2 in float64, one workgroup.
__global__ __launch_bounds__(256) void k_mlp_loss(const float *__restrict__ y,
                                                  const float *__restrict__ t, int batch,
                                                  double *__restrict__ out) {
    __shared__ double red[4];
    double s = 0.0;
    for (int k = threadIdx.x; k < batch * NO; k += 256) {
        const double d = (double)y[k] - (double)t[k];
        s += d * d;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = (red[0] + red[1] + red[2] + red[3]) * 0.5 / (double)batch;
}

// Adam with bias correction; c1 = 1 - beta1^t, c2 = 1 - beta2^t (host).
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float beta1, float beta2,
                       float eps, float c1, float c2) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = fmaf(beta1, m[k], (1.0f - beta1) * gk);
    const float vk = fmaf(beta2, v[k], (1.0f - beta2) * gk * gk);
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// Row statistics of a float64 block-CSR matrix relative to an interval
// centre c and half width w: per scalar row r, d~ = (H_rr - c) / w and
// R~ = sum_{s != r} |H_rs| / w.  Integer histograms (d~ over [-1, 1] in
// kDiagBins bins, R~ over [0, 1] in kRadBins bins, clamped) and per-workgroup
// partials {sum d~, sum d~^2, sum R~, max R~, min d~, max d~}.
__global__ __launch_bounds__(256) void k_row_features(int b, int nb, const int64_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci,
                                                      const double *__restrict__ val, double c,
                                                      double w, uint32_t *__restrict__ hist,
                                                      double *__restrict__ part) {
    __shared__ double sm[6][4];
    const int64_t n = (int64_t)nb * b;
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double sd = 0, sd2 = 0, sr = 0, mr = -1e300, mnd = 1e300, mxd = -1e300;
    if (r < n) {
        const int I = (int)(r / b), rr = (int)(r % b);
        double d = 0.0, R = 0.0;
        for (int64_t k = rp[I]; k < rp[I + 1]; ++k) {
            const double *blk = val + (k * b + rr) * b;
            const bool diag = ci[k] == I;
            for (int s = 0; s < b; ++s) {
                if (diag && s == rr)
                    d = blk[s];
                else
                    R += fabs(blk[s]);
            }
        }
        const double dt = (d - c) / w, rt = R / w;
        int bd = (int)floor((dt + 1.0) * 0.5 * kDiagBins);
        bd = bd < 0 ? 0 : (bd >= kDiagBins ? kDiagBins - 1 : bd);
        int br = (int)floor(rt * kRadBins);
        br = br < 0 ? 0 : (br >= kRadBins ? kRadBins - 1 : br);
        atomicAdd(&hist[bd], 1u);
        atomicAdd(&hist[kDiagBins + br], 1u);
        sd = dt;
        sd2 = dt * dt;
        sr = rt;
        mr = rt;
        mnd = dt;
        mxd = dt;
    }
    for (int off = 32; off > 0; off >>= 1) {
        sd += __shfl_xor(sd, off, 64);
        sd2 += __shfl_xor(sd2, off, 64);
        sr += __shfl_xor(sr, off, 64);
        mr = fmax(mr, __shfl_xor(mr, off, 64));
        mnd = fmin(mnd, __shfl_xor(mnd, off, 64));
        mxd = fmax(mxd, __shfl_xor(mxd, off, 64));
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sm[0][wv] = sd;
        sm[1][wv] = sd2;
        sm[2][wv] = sr;
        sm[3][wv] = mr;
        sm[4][wv] = mnd;
        sm[5][wv] = mxd;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double o[6] = {sm[0][0], sm[1][0], sm[2][0], sm[3][0], sm[4][0], sm[5][0]};
        for (int q = 1; q < 4; ++q) {
            o[0] += sm[0][q];
            o[1] += sm[1][q];
            o[2] += sm[2][q];
            o[3] = fmax(o[3], sm[3][q]);
            o[4] = fmin(o[4], sm[4][q]);
            o[5] = fmax(o[5], sm[5][q]);
        }
        for (int q = 0; q < 6; ++q) part[(size_t)blockIdx.x * 6 + q] = o[q];
    }
}

}  // namespace

hipError_t launch_mlp_forward(const float *params, const float *norm, const float *x, int batch,
                              float *hid, float *y, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3(batch), dim3(NH), 0, st, params, norm, x, batch, hid, y);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *params, const float *x, const float *hid, const float *y,
                           const float *t, int batch, float *dy, float *dh, float *grad,
                           double *loss, hipStream_t st) {
    if (batch <= 0) return hipErrorInvalidValue;
    const int64_t nd = (int64_t)batch * NH;
    hipLaunchKernelGGL(k_mlp_delta, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, st, params,
                       hid, y, t, batch, dy, dh);
    hipLaunchKernelGGL(k_mlp_grad, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, x, hid, dy,
                       dh, batch, grad);
    if (loss) hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, st, y, t, batch, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                       float beta1, float beta2, float eps, float c1, float c2, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, g, m, v, n,
                       lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError();
}

int row_feature_parts(int b, int nb) { return (int)(((int64_t)nb * b + 255) / 256); }

hipError_t launch_row_features(int b, int nb, const int64_t *rp, const int32_t *ci,
                               const double *val, double c, double w, uint32_t *hist,
                               double *part, hipStream_t st) {
    hipLaunchKernelGGL(k_row_features, dim3(row_feature_parts(b, nb)), dim3(256), 0, st, b, nb, rp,
                       ci, val, c, w, hist, part);
    return hipGetLastError();
}

}  // namespace chess

// ---------------------------------------------------------------------------
// Allocation-free gradient (chess_mlp_grad_noalloc): its workspace is this
// fixed array - one float64 loss at offset 0, then dy [batch][3] and
// dh [batch][128] floats from offset 256 - for batches of at most
// CHESS_NOALLOC_MAX_BATCH rows.  Every GPU that runs the library holds its
// own copy until the process ends; in host code `scratch` names a host-side
// stand-in, so its device address is taken once per device (with that device
// current) by noalloc_scratch_init and used everywhere instead of the name.
// The kernels write every workspace value before reading it, so nothing needs
// clearing between calls; calls that overlap on one GPU share it and race.
// ---------------------------------------------------------------------------
namespace chess {
namespace {
constexpr size_t kNoAllocBytes =
    256 + (size_t)CHESS_NOALLOC_MAX_BATCH * (kMlpOut + kMlpHidden) * sizeof(float);
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;
}  // namespace
}  // namespace chess

static __device__ __align__(256) unsigned char scratch[chess::kNoAllocBytes];

namespace chess {

hipError_t noalloc_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

}  // namespace chess

extern "C" int chess_mlp_grad_noalloc(chess_ctx *ctx, const float *params, const float *x,
                                      const float *hidden, const float *y, const float *target,
                                      int32_t batch, float *grad, double *loss) {
    using namespace chess;
    if (!ctx) return CHESS_E_ARG;
    if (!params || !x || !hidden || !y || !target || !grad || batch <= 0) {
        ctx_set_error(ctx, "mlp_grad_noalloc: null pointer or empty batch");
        return CHESS_E_ARG;
    }
    if (batch > CHESS_NOALLOC_MAX_BATCH) {
        ctx_set_error(ctx, "mlp_grad_noalloc: batch exceeds CHESS_NOALLOC_MAX_BATCH (the fixed workspace)");
        return CHESS_E_ARG;
    }
    const int dev = ctx_device(ctx);
    hipStream_t st = ctx_stream(ctx);
    hipError_t e = hipSetDevice(dev);
    void *base = nullptr;
    if (e == hipSuccess) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr;
    }
    if (e != hipSuccess || !base) {
        ctx_set_error(ctx, "mlp_grad_noalloc: no workspace address for this device");
        return CHESS_E_HIP;
    }
    double *dl = static_cast<double *>(base);
    float *dy = reinterpret_cast<float *>(static_cast<unsigned char *>(base) + 256);
    float *dh = dy + (size_t)batch * kMlpOut;
    e = launch_mlp_grad(params, x, hidden, y, target, batch, dy, dh, grad, loss ? dl : nullptr, st);
    if (e == hipSuccess && loss) {
        e = hipMemcpyAsync(loss, dl, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    if (e != hipSuccess) {
        ctx_set_error(ctx, hipGetErrorString(e));
        return CHESS_E_HIP;
    }
    ctx_set_error(ctx, "no error");
    return CHESS_OK;
}
