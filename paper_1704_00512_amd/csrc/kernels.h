// Internal interface between the host pipeline (chess.cpp) and the HIP
// kernels (kernels.hip).  Not part of the public C interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef struct chess_ctx chess_ctx;

namespace chess {

// Symbolic plan of one masked block product C = P_C o (A Bt^T), all three in
// block CSR.  Output block rows are grouped into tiles of consecutive rows;
// a tile's rows of A are staged in LDS.  For every tile:
//   u list: the distinct column indices of A over the tile's rows (sorted),
//           with, per tile row i, the block's position inside the staged A
//           tile (0xFFFF if row i has no such column);
//   j list: the distinct column indices of C over the tile's rows (sorted),
//           with, per tile row i, the block's offset inside C's row (0xFFFF
//           if absent).
struct ProductPlanDev {
    int ntiles = 0;
    int cmax = 0;          // rows per tile upper bound (kernel template value)
    int hcap_log2 = 0;     // LDS hash table size = 1 << hcap_log2
    int lds_ablocks = 0;   // largest A tile in blocks
    int max_u = 0;         // largest u list
    int max_bt_row = 0;    // longest row of Bt (per-wave LDS staging)
    int stage_bt = 0;      // 1: each wave copies its Bt row to LDS first
    const int32_t *tile_row0 = nullptr;  // [ntiles + 1]
    const int64_t *u_off = nullptr;      // [ntiles + 1]
    const int32_t *u_cols = nullptr;
    const uint16_t *u_pos = nullptr;     // [total_u * cmax]
    const int64_t *j_off = nullptr;      // [ntiles + 1]
    const int32_t *j_cols = nullptr;
    const uint16_t *j_pos = nullptr;     // [total_j * cmax]
    const int32_t *j_rec = nullptr;      // [total_j * 4]: j, Bt row start, Bt row length, 0
};

// Epilogue applied to Y = P_C o (A Bt^T) at every output element:
//   out = alpha * Y + beta * prev          (prev may be null: beta ignored)
//   out is stored to `out` (may alias prev: each element is read then written
//   by the same thread);
//   acc[q] += coef[q] * out in float64 for q < nacc;
//   hist (if set) receives a copy of out;
//   trace_partial (if set) receives, per tile, the float64 sum of out over
//   the diagonal elements of diagonal blocks.
struct Epilogue {
    double alpha = 1.0, beta = 0.0;
    const void *prev = nullptr;
    int nacc = 0;
    double *acc[4] = {nullptr, nullptr, nullptr, nullptr};
    double coef[4] = {0, 0, 0, 0};
    void *hist = nullptr;
    double *trace_partial = nullptr;
    // batches of systems (listed and searching kernels): when row_sys is set, the
    // weight of accumulator q for a tile is coef_sys[q][row_sys[first row]]
    // (tiles never straddle systems) instead of coef[q]
    const int32_t *row_sys = nullptr;
    const double *coef_sys[4] = {nullptr, nullptr, nullptr, nullptr};
    // batches: the last chain step each system needs (sys_last[s]) and the
    // step of this launch; the tiles of a system past its last step return
    // at once (their T, sums and moments are no longer read)
    const int32_t *sys_last = nullptr;
    int step = 0;
    // moments-only chains (output-stationary kernel only): per tile, the
    // Frobenius products <Y', Y'> and <Y', A> of the finished output Y' with
    // A (the chain's T_m, stored on the output's pattern), float64
    double *sq_partial = nullptr;
    double *xy_partial = nullptr;
};

// True when this tile's system needs no more chain steps (see Epilogue); the
// caller returns, after its trace partial is set to 0.
__device__ inline bool tile_finished(const Epilogue &ep, int tile, int row0) {
    if (!ep.sys_last || !ep.row_sys || ep.step <= ep.sys_last[ep.row_sys[row0]]) return false;
    if (threadIdx.x == 0 && ep.trace_partial) ep.trace_partial[tile] = 0.0;
    return true;
}

struct ProductOperands {
    const int64_t *a_rp;
    const void *a_val;
    const int64_t *bt_rp;
    const int32_t *bt_ci;
    const void *bt_val;
    const int64_t *c_rp;
    void *c_out;
    // bfloat16 operand forms of Bt (output-stationary kernel, kStatBF16 and
    // kStatBF16X3): hi = bf16(x), lo = bf16(x - hi), same block layout
    const void *bt_hi = nullptr;
    const void *bt_lo = nullptr;
    // operand mode of the product: 0 = the storage precision (dtype);
    // kStatBF16 or kStatBF16X3 (float32 storage, output-stationary kernel only)
    int opmode = 0;
};

// Operand modes of the output-stationary product (kernels_stat.hip)
enum { kStatF32 = 0, kStatBF16 = 1, kStatBF16X3 = 2, kStatF64 = 3 };

// Plan of a product with precomputed hit lists (kernels_listed.hip).  Per
// tile the output columns j; per column a record of 8 int32:
//   {j, Bt row start, Bt row length, first entry,
//    hit counts of tile rows 0..3 (8 bits each), out pos rows 0|1, 2|3, 0}
// where "out pos" is the block's offset in the output row (0xFFFF: absent).
// Entries (entry_width 1: 8-bit position in A row i | 8-bit position in Bt
// row j << 8; entry_width 2: 16 + 16 bits) are grouped per column, row 0's
// hits first; every column's group starts on a 4-byte boundary.
struct ListedPlanDev {
    int ntiles = 0;
    int cmax = 0;
    int lds_ablocks = 0;
    int max_bt_row = 0;
    int max_entries = 0;
    int entry_width = 1;
    // kernel variant (MFMA paths only; others have variant 0 alone):
    //   0: Bt rows staged in LDS, 8 waves (float) / 4 waves (double)
    //   1: Bt operands read from global memory, same wave count
    //   2: Bt operands from global memory, twice the waves
    //   3: Bt operands from global memory, half the waves
    //   4, 5 (float32 only): as 1 and 2 with the hit groups software-pipelined
    //   6, 7: as 1 and 2 with non-temporal hints on the streamed data
    //   8, 9: as 1 and 2 with all operand loads of a hit group issued before
    //      its MFMAs (scheduling barrier)
    //   10, 11 / 12, 13 (float32 only): as 8 and 9 with 6 / 8 hits per slot
    //      per group and two accumulators (8 hits: LDS reads after the barrier)
    //   14 / 15 (float32 only): as 12 / 10 with the last group padded past
    //      the lists (one wait per group, no remainder loops)
    //   16-19 (float32 only, plans with lean_rec): the 16 MFMA slots shared
    //      freely among the tile rows (k_lean); 8 waves with 8-round groups,
    //      12 waves with 8-round groups, 8 waves with 4-round groups, 16 waves
    //      with 4-round groups
    //   20-22: as 16, 18, 19 with the next column's loads issued after the
    //      last group's Bt loads; 23: as 21 with 10 waves (<= 96 VGPRs)
    // float32, b = 9 (tiles of 2 rows): 0 vector ALU; 1, 2: MFMA (k_listed9)
    //   with 4 or 8 waves; 3, 4: MFMA with pipelined columns (k_lean9), 8 or
    //   4 waves
    int variant = 0;
    const int32_t *tile_row0 = nullptr;  // [ntiles + 1]
    const int64_t *j_off = nullptr;      // [ntiles + 1]
    const int32_t *j_rec = nullptr;      // [total_j * 8]
    const void *entries = nullptr;
    // Free slot assignment (float32, b = 4; null otherwise): per column a
    // record of 8 int32 {j, Bt row start, Bt row length, first round,
    // R | n_0 << 8 | n_1 << 13 | n_2 << 18 | n_3 << 23, out pos rows 0|1,
    // 2|3, 0}: R rounds (even, <= 32) of the 16 MFMA slots, tile row i on n_i
    // consecutive slots (sum <= 16).  Per round 32 bytes: the position in
    // A row i of each slot's hit, then its position in Bt row j (255 past
    // the slot's list).
    const int32_t *lean_rec = nullptr;
    const uint8_t *lean_ent = nullptr;
    int max_cols = 0;  // most output columns of a tile
    // element offsets of the output pattern (in float64) and byte offsets of
    // the hit lists fit in 31 bits (buffer-descriptor addressing)
    bool off31 = false;
    // Output-stationary plan (b = 4; null otherwise): the output blocks of
    // tile t, sorted by hit count, form the groups [st_goff[t], st_goff[t+1])
    // of st_g slots.  Per group st_ginfo {list offset in 16-byte units,
    // R | diagonal-slot mask << 16} with R (rounds) a multiple of 8; per group
    // and slot st_slot {output block (0xFFFFFFFF: none), Bt row start block |
    // A row start block in the LDS tile << 22}; per slot a list of R two-byte
    // entries (position in A row | position in Bt row << 8), padded with the
    // row's zero block (position = row length).  In LDS each tile row is
    // followed by one zero block (st_ablocks: the largest tile so laid out).
    const int32_t *st_goff = nullptr;
    const int32_t *st_ginfo = nullptr;
    const uint32_t *st_slot = nullptr;
    const void *st_list = nullptr;
    int st_g = 0;
    int st_ablocks = 0;
};

// The output-stationary product (kernels_stat.hip): mode kStat*, nw waves
// per workgroup (4, 8 or 16).  lds_out (if not null) receives the LDS bytes
// and nothing is launched.
hipError_t launch_stat_product(int mode, int nw, const ListedPlanDev &plan, const ProductOperands &ops,
                               const Epilogue &ep, hipStream_t st, size_t *lds_out);
// hi[i] = bf16(in[i]), lo[i] = bf16(in[i] - hi[i]) (lo may be null)
hipError_t launch_split_bf16(int64_t n, const float *in, unsigned short *hi, unsigned short *lo, hipStream_t st);

hipError_t launch_listed_product(int dtype, int b, const ListedPlanDev &plan,
                                 const ProductOperands &ops, const Epilogue &ep, hipStream_t st);
size_t listed_product_lds_bytes(int dtype, int b, const ListedPlanDev &plan, int opmode = 0);
// number of kernel variant ids for this dtype / b / plan.cmax (>= 1), and
// whether id v exists
int listed_product_variants(int dtype, int b, const ListedPlanDev &plan);
bool listed_product_variant_ok(int dtype, int b, const ListedPlanDev &plan, int v, int opmode = 0);
// variant ids of the output-stationary kernel: float32 storage 24, 25, 26
// (8, 4, 16 waves; also the ids for the bfloat16 operand modes), float64
// storage 10, 11, 12 (4, 8, 16 waves)
constexpr int kStatVariantF32 = 24, kStatVariantF64 = 10;

// Context accessors for entry points outside chess.cpp (chess_ctx is opaque
// there), and the per-device workspace address of chess_mlp_grad_noalloc
// (learned.hip), taken once per device when a context is created.
int ctx_device(const chess_ctx *ctx);
hipStream_t ctx_stream(const chess_ctx *ctx);
void ctx_set_error(chess_ctx *ctx, const char *msg);
hipError_t noalloc_scratch_init(int device);

// Learned predictor (learned.hip): perceptron sizes, feature histograms.
constexpr int kMlpIn = 64, kMlpHidden = 128, kMlpOut = 3;
constexpr int kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + kMlpOut * kMlpHidden + kMlpOut;
constexpr int kMlpNorm = 2 * kMlpIn + 2 * kMlpOut;
constexpr int kDiagBins = 24, kRadBins = 16;
// y [batch][3] = net(x [batch][64]); hid [batch][128] (tanh outputs) if not null
hipError_t launch_mlp_forward(const float *params, const float *norm, const float *x, int batch,
                              float *hid, float *y, hipStream_t st);
// grad = dL/dparams for targets t; dy [batch][3], dh [batch][128] are scratch;
// loss (device float64, may be null) = L
hipError_t launch_mlp_grad(const float *params, const float *x, const float *hid, const float *y,
                           const float *t, int batch, float *dy, float *dh, float *grad,
                           double *loss, hipStream_t st);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                       float beta1, float beta2, float eps, float c1, float c2, hipStream_t st);
// hist (kDiagBins + kRadBins uint32, zeroed by the caller); part [parts][6]
int row_feature_parts(int b, int nb);
hipError_t launch_row_features(int b, int nb, const int64_t *rp, const int32_t *ci,
                               const double *val, double c, double w, uint32_t *hist,
                               double *part, hipStream_t st);

// dtype: 0 = double, 1 = float.  Returns a hipError_t.
hipError_t launch_masked_product(int dtype, int b, const ProductPlanDev &plan,
                                 const ProductOperands &ops, const Epilogue &ep,
                                 hipStream_t st);
size_t masked_product_lds_bytes(int dtype, int b, const ProductPlanDev &plan);

// Elementwise and small kernels (all on block-CSR value arrays, nb = blocks).
hipError_t launch_fill_identity(int dtype, int b, int64_t nnzb, const int32_t *brow,
                                const int32_t *bcol, void *out, hipStream_t st);
// out[map[p]] = transpose_if(in[p]) (converted to dtype_out); out must be zeroed
// first when the map does not cover it.
hipError_t launch_scatter_blocks(int dtype_out, int b, int64_t nnzb_in, const int64_t *map,
                                 const double *in, void *out, int transpose, hipStream_t st);
// out = sigma * (in - tau I) (float64, same pattern)
hipError_t launch_scale_shift(int b, int64_t nnzb, const int32_t *brow, const int32_t *bcol,
                              const double *in, double *out, double sigma, double tau,
                              hipStream_t st);
// same with sigma[row_sys[I]] and tau[row_sys[I]] per block row I
hipError_t launch_scale_shift_rows(int b, int64_t nnzb, const int32_t *brow, const int32_t *bcol,
                                  const int32_t *row_sys, const double *sigma, const double *tau,
                                  const double *in, double *out, hipStream_t st);
// out[k * nseg + s] = sum_{t in [seg[s], seg[s+1])} part[k * ntiles + t], k < nk
hipError_t launch_segment_sum(int nk, int ntiles, int nseg, const int32_t *seg, const double *part,
                              double *out, hipStream_t st);
// out[p] = 0.5 (in[p] + in[tmap[p]]^T)
hipError_t launch_symmetrize(int b, int64_t nnzb, const int64_t *tmap, const double *in,
                             double *out, hipStream_t st);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);
// acc = a0 * T0 + a1 * T1 (T in dtype, acc float64)
hipError_t launch_axpby_to_f64(int dtype, int64_t n, double a0, const void *t0, double a1,
                               const void *t1, double *acc, hipStream_t st);
// acc[x] = sum_k coef[k] hist[k][x] for k < nk (coef on device)
hipError_t launch_recombine(int dtype, int64_t n, int nk, const void *hist, const double *coef,
                            double *acc, hipStream_t st);
// Per block row diagonal trace partials, reduced per tile of rows.
hipError_t launch_trace(int dtype, int b, int nb, const int64_t *diag_idx, const void *val,
                        double *out_partial, int nparts, hipStream_t st);
// Partials of the Frobenius products <x, x> (part[0 .. nparts)) and <x, y>
// (part[nparts .. 2 nparts)) of two value arrays of n entries, 16-byte aligned.
hipError_t launch_dot_pair(int dtype, int64_t n, const void *x, const void *y, double *part,
                           int nparts, hipStream_t st);
// out[s] = sum_t part[s * nparts + t], fixed order.
hipError_t launch_reduce_rows(int nrows, int nparts, const double *part, double *out,
                              hipStream_t st);
// Gershgorin: per scalar row d - R and d + R, reduced to per-tile min/max.
hipError_t launch_gershgorin(int b, int nb, const int64_t *rp, const int32_t *ci,
                             const double *val, double *part_lo, double *part_hi, int nparts,
                             hipStream_t st);
hipError_t launch_minmax(int nparts, const double *part_lo, const double *part_hi, double *out2,
                         hipStream_t st);
// y = A x (block CSR, float64)
hipError_t launch_spmv(int b, int nb, const int64_t *rp, const int32_t *ci, const double *val,
                       const double *x, double *y, hipStream_t st);
// h[j] = V[j] . w for j < m (V row-major [m][n]) ; partials per tile
hipError_t launch_multidot(int m, int64_t n, const double *V, const double *w, double *part,
                           int nparts, hipStream_t st);
// w -= sum_j h[j] V[j]
hipError_t launch_multiaxpy(int m, int64_t n, const double *V, const double *h, double *w,
                            hipStream_t st);
// y = x * s (s read from device scalar: y = x / sqrt(*nrm2))
hipError_t launch_normalize(int64_t n, const double *x, const double *nrm2, double *y,
                            hipStream_t st);
// sum over S blocks q of sum_rs K[kmap[q]][r][s] * S[q][s][r]  (Tr(K S)) partials
hipError_t launch_trace_product(int b, int64_t nnzb_s, const int64_t *kmap_t, const double *K,
                                const double *S, double *part, int nparts, hipStream_t st);
hipError_t launch_convert(int dtype_out, int64_t n, const double *in, void *out, hipStream_t st);

}  // namespace chess
