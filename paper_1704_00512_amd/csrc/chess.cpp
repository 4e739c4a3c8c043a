// Host pipeline behind the C interface of include/chess.h.
//
// Flow of chess_fermi_operator (Sec. "Fermi Operator Expansion"):
//   patterns  -> validated host copies, transpose and embedding maps, and
//                cached symbolic product plans (integer work, once per pattern)
//   S bounds  -> Gershgorin upper bound, Lanczos lower bound (GPU SpMV)
//   X^T       -> Chebyshev chain on S~ with f = x^-1/2 (Sec. "Matrix powers")
//   H'        -> P_H o (X P_K o (H X)), symmetrised (two masked products)
//   bounds    -> Gershgorin or Lanczos on H', checked afterwards by Eq. 6
//   n_pl      -> Eq. 7 at mu = tau
//   chain     -> Chebyshev chain on H~' with trace moments (and, optionally,
//                every T_k kept for recombination)
//   mu        -> bisection on N(mu) from the moments (host)
//   K'        -> recombination of the kept T_k, or a second chain pass
//   K         -> P_K o (X P_K o (K' X)), Tr(KS)
//
// All device work is on the context stream; host decisions (bounds, degree,
// mu) read back a handful of doubles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/chess.h"
#include "hostmath.h"
#include "kernels.h"

namespace chess {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

struct Error {
    int code;
    std::string msg;
};

#define CHESS_THROW(code, ...)                                  \
    do {                                                        \
        char _buf[512];                                         \
        std::snprintf(_buf, sizeof(_buf), __VA_ARGS__);         \
        throw Error{code, std::string(_buf)};                   \
    } while (0)

#define HIPCHECK(expr)                                                                    \
    do {                                                                                  \
        hipError_t _e = (expr);                                                           \
        if (_e != hipSuccess)                                                             \
            CHESS_THROW(_e == hipErrorOutOfMemory ? CHESS_E_OOM : CHESS_E_HIP, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(_e), __FILE__, __LINE__);                \
    } while (0)

// ---------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    explicit DevBuf(size_t n) { alloc(n); }
    void alloc(size_t n) {
        release();
        if (n == 0) n = 16;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            CHESS_THROW(CHESS_E_OOM, "hipMalloc(%zu bytes) failed: %s", n, hipGetErrorString(e));
        }
        bytes = n;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    ~DevBuf() { release(); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    template <typename T>
    T *as() const { return reinterpret_cast<T *>(p); }
};

template <typename T>
static void upload(DevBuf &d, const std::vector<T> &h, hipStream_t st) {
    d.alloc(h.size() * sizeof(T));
    if (!h.empty()) HIPCHECK(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

// ---------------------------------------------------------------------------
// patterns
// ---------------------------------------------------------------------------

struct Pattern {
    int b = 0;
    int nb = 0;
    int64_t nnzb = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<int64_t> tmap;  // index of block (j, i) for block p = (i, j)
    std::vector<int64_t> diag;  // index of block (i, i)
    int max_row = 0;
    DevBuf d_rp, d_ci, d_brow, d_diag, d_tmap;
    int64_t n() const { return (int64_t)nb * b; }
    int64_t find(int i, int j) const {
        auto beg = ci.begin() + rp[i], end = ci.begin() + rp[i + 1];
        auto it = std::lower_bound(beg, end, j);
        if (it == end || *it != j) return -1;
        return (int64_t)(it - ci.begin());
    }
};

struct EmbedMap {
    const Pattern *from = nullptr, *to = nullptr;
    std::vector<int64_t> map;    // position in `to` of each block of `from`
    DevBuf d_map, d_map_t;       // map, and map of the transposed block
};

struct ProductPlan {
    const Pattern *a = nullptr, *bt = nullptr, *c = nullptr;
    int dtype = 0;
    std::vector<int32_t> breaks;     // rows where a tile must start (batches: system starts)
    std::vector<int32_t> tile_row0;  // host copy, ntiles + 1
    ProductPlanDev dev;
    DevBuf d_tile_row0, d_u_off, d_u_cols, d_u_pos, d_j_off, d_j_cols, d_j_pos, d_j_rec;
};

// Product with precomputed hit lists (kernels_listed.hip), for chains.
struct ListedPlan {
    const Pattern *a = nullptr, *bt = nullptr, *c = nullptr;
    int dtype = 0;
    int cmax = 0;         // rows per tile (at most)
    bool usable = false;  // false: rows too long for the list format
    // fastest kernel variant per operand mode, for passes without and with
    // float64 sums (-1: not timed yet)
    int tuned_variant[3][2] = {{-1, -1}, {-1, -1}, {-1, -1}};
    double tuned_ms[3][2] = {{-1, -1}, {-1, -1}, {-1, -1}};  // its time per product
    std::vector<int32_t> breaks;     // rows where a tile must start (batches: system starts)
    std::vector<int32_t> tile_row0;  // host copy, ntiles + 1
    ListedPlanDev dev;
    DevBuf d_tile_row0, d_j_off, d_j_rec, d_entries, d_lean_rec, d_lean_ent;
    DevBuf d_st_goff, d_st_ginfo, d_st_slot, d_st_list;  // output-stationary groups
};

// Learned bound / mu predictor loaded by chess_model_load (layout of the
// blob: see CHESS_MODEL_FLOATS in chess.h).
struct Model {
    bool loaded = false;
    std::vector<float> blob;
    DevBuf norm, params;
    double margin_lo = 0, margin_hi = 0, mu_half = 0;  // in Gershgorin half widths
};

}  // namespace chess

struct chess_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err = "no error";
    std::vector<std::unique_ptr<chess::Pattern>> patterns;
    std::vector<std::unique_ptr<chess::EmbedMap>> embeds;
    std::vector<std::unique_ptr<chess::ProductPlan>> plans;
    std::vector<std::unique_ptr<chess::ListedPlan>> lplans;
    // tile heights chosen by timing, per (A, Bt, storage, system breaks,
    // operand mode, pass with or without float64 sums)
    struct TileChoice {
        const chess::Pattern *a, *bt;
        int dtype;
        std::vector<int32_t> breaks;
        int opmode, pass, rows;
    };
    std::vector<TileChoice> tile_choices;
    chess_progress_fn progress = nullptr;
    void *progress_user = nullptr;
    int32_t progress_every = 0;
    chess::Model model;
    chess::DevBuf loss_buf;  // one float64: loss of chess_mlp_grad
    hipStream_t capture_stream = nullptr;  // records graphs (not the null stream)
};

namespace chess {

static void validate_pattern_struct(const chess_pattern *p, const char *what) {
    if (!p) CHESS_THROW(CHESS_E_ARG, "%s: null pattern", what);
    if (p->b != 4 && p->b != 9) CHESS_THROW(CHESS_E_UNSUPPORTED, "%s: block edge %d (4 or 9 supported)", what, p->b);
    if (p->nbrows <= 0 || p->nnzb < p->nbrows) CHESS_THROW(CHESS_E_ARG, "%s: nbrows %d, nnzb %lld", what, p->nbrows, (long long)p->nnzb);
    if (!p->row_ptr || !p->col_idx) CHESS_THROW(CHESS_E_ARG, "%s: null row_ptr/col_idx", what);
}

// Copies a caller pattern to the host, validates it and returns the cached
// entry with identical content (or a new one).
static const Pattern *get_pattern_host(chess_ctx *ctx, int b, int nbrows, int64_t nnzb,
                                       std::vector<int64_t> rp, std::vector<int32_t> ci,
                                       const char *what) {
    hipStream_t st = ctx->stream;
    for (auto &e : ctx->patterns) {
        if (e->b == b && e->nb == nbrows && e->nnzb == nnzb && e->rp == rp && e->ci == ci)
            return e.get();
    }
    auto P = std::make_unique<Pattern>();
    P->b = b;
    P->nb = nbrows;
    P->nnzb = nnzb;
    if (rp[0] != 0 || rp[nbrows] != nnzb) CHESS_THROW(CHESS_E_PATTERN, "%s: row_ptr must start at 0 and end at nnzb", what);
    P->diag.assign(nbrows, -1);
    for (int i = 0; i < nbrows; ++i) {
        if (rp[i + 1] < rp[i]) CHESS_THROW(CHESS_E_PATTERN, "%s: row_ptr decreases at row %d", what, i);
        P->max_row = std::max<int>(P->max_row, (int)(rp[i + 1] - rp[i]));
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
            const int j = ci[q];
            if (j < 0 || j >= nbrows) CHESS_THROW(CHESS_E_PATTERN, "%s: column %d out of range in row %d", what, j, i);
            if (q > rp[i] && ci[q - 1] >= j) CHESS_THROW(CHESS_E_PATTERN, "%s: columns not strictly increasing in row %d", what, i);
            if (j == i) P->diag[i] = q;
        }
        if (P->diag[i] < 0) CHESS_THROW(CHESS_E_PATTERN, "%s: diagonal block missing in row %d", what, i);
    }
    P->rp = std::move(rp);
    P->ci = std::move(ci);
    P->tmap.assign((size_t)nnzb, -1);
    std::vector<int32_t> brow((size_t)nnzb);
    for (int i = 0; i < nbrows; ++i) {
        for (int64_t q = P->rp[i]; q < P->rp[i + 1]; ++q) {
            brow[q] = i;
            const int64_t t = P->find(P->ci[q], i);
            if (t < 0) CHESS_THROW(CHESS_E_PATTERN, "%s: pattern not symmetric at block (%d, %d)", what, i, P->ci[q]);
            P->tmap[q] = t;
        }
    }
    upload(P->d_rp, P->rp, st);
    upload(P->d_ci, P->ci, st);
    upload(P->d_brow, brow, st);
    upload(P->d_diag, P->diag, st);
    upload(P->d_tmap, P->tmap, st);
    HIPCHECK(hipStreamSynchronize(st));
    ctx->patterns.push_back(std::move(P));
    return ctx->patterns.back().get();
}

static const Pattern *get_pattern(chess_ctx *ctx, const chess_pattern *p, const char *what) {
    validate_pattern_struct(p, what);
    hipStream_t st = ctx->stream;
    std::vector<int64_t> rp((size_t)p->nbrows + 1);
    std::vector<int32_t> ci((size_t)p->nnzb);
    HIPCHECK(hipMemcpyAsync(rp.data(), p->row_ptr, rp.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(ci.data(), p->col_idx, ci.size() * 4, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    return get_pattern_host(ctx, p->b, p->nbrows, p->nnzb, std::move(rp), std::move(ci), what);
}

static const EmbedMap *get_embed(chess_ctx *ctx, const Pattern *from, const Pattern *to,
                                 const char *what) {
    for (auto &e : ctx->embeds)
        if (e->from == from && e->to == to) return e.get();
    if (from->nb != to->nb || from->b != to->b) CHESS_THROW(CHESS_E_ARG, "%s: patterns differ in size", what);
    auto E = std::make_unique<EmbedMap>();
    E->from = from;
    E->to = to;
    E->map.resize((size_t)from->nnzb);
    std::vector<int64_t> mt((size_t)from->nnzb);
    for (int i = 0; i < from->nb; ++i) {
        for (int64_t q = from->rp[i]; q < from->rp[i + 1]; ++q) {
            const int64_t p = to->find(i, from->ci[q]);
            if (p < 0) CHESS_THROW(CHESS_E_PATTERN, "%s: block (%d, %d) not in the larger pattern", what, i, from->ci[q]);
            E->map[q] = p;
        }
    }
    for (int64_t q = 0; q < from->nnzb; ++q) mt[q] = E->map[from->tmap[q]];
    upload(E->d_map, E->map, ctx->stream);
    upload(E->d_map_t, mt, ctx->stream);
    HIPCHECK(hipStreamSynchronize(ctx->stream));
    ctx->embeds.push_back(std::move(E));
    return ctx->embeds.back().get();
}

static int pick_cmax(int dtype, int b) {
    if (b == 4) return 4;
    return dtype == 1 ? 2 : 1;
}

// Chain storage precision (0 = float64, 1 = float32) and operand mode of the
// products (kernels.h) for an opts precision: the bfloat16 forms keep T_k in
// float32 and round only the product operands.
static int storage_dtype(int precision) { return precision == CHESS_F64 ? 0 : 1; }
static int operand_mode(int precision) {
    return precision == CHESS_BF16 ? kStatBF16 : precision == CHESS_BF16X3 ? kStatBF16X3 : 0;
}

// Symbolic plan of C = P_C o (A Bt^T) (see kernels.h); tiles start at every
// row in `breaks` (batches: the first row of each system).
static const ProductPlan *get_plan(chess_ctx *ctx, const Pattern *A, const Pattern *Bt,
                                   const Pattern *C, int dtype, const std::vector<int32_t> &breaks = {}) {
    for (auto &e : ctx->plans)
        if (e->a == A && e->bt == Bt && e->c == C && e->dtype == dtype && e->breaks == breaks) return e.get();
    auto P = std::make_unique<ProductPlan>();
    P->a = A;
    P->bt = Bt;
    P->c = C;
    P->dtype = dtype;
    P->breaks = breaks;
    std::vector<char> is_break(A->nb + 1, 0);
    for (int32_t r : breaks)
        if (r >= 0 && r <= A->nb) is_break[r] = 1;
    const int b = A->b;
    const int cmax = pick_cmax(dtype, b);
    const size_t block_bytes = (size_t)b * b * (dtype == 1 ? 4 : 8);
    // LDS budget for the staged A tile: 48 KB (float32) or 80 KB (float64)
    const size_t a_budget = dtype == 1 ? 49152 : 81920;
    const int budget_blocks = std::max<int>((int)(a_budget / block_bytes), A->max_row);
    std::vector<int32_t> tile_row0;
    std::vector<int64_t> u_off{0}, j_off{0};
    std::vector<int32_t> u_cols, j_cols;
    std::vector<uint16_t> u_pos, j_pos;
    int lds_ablocks = 0, max_u = 0;
    int r = 0;
    std::vector<int32_t> merged;
    while (r < A->nb) {
        const int row0 = r;
        int64_t blocks = 0;
        while (r < A->nb && r - row0 < cmax) {
            const int64_t len = A->rp[r + 1] - A->rp[r];
            if (r > row0 && (blocks + len > budget_blocks || is_break[r])) break;
            blocks += len;
            ++r;
        }
        const int c = r - row0;
        tile_row0.push_back(row0);
        lds_ablocks = std::max<int>(lds_ablocks, (int)blocks);
        if (blocks >= 0xFFFF) CHESS_THROW(CHESS_E_UNSUPPORTED, "row tile of %lld blocks is too long", (long long)blocks);
        // u list
        merged.assign(A->ci.begin() + A->rp[row0], A->ci.begin() + A->rp[r]);
        std::sort(merged.begin(), merged.end());
        merged.erase(std::unique(merged.begin(), merged.end()), merged.end());
        const size_t ubase = u_cols.size();
        u_cols.insert(u_cols.end(), merged.begin(), merged.end());
        u_pos.resize(u_cols.size() * cmax, 0xFFFF);
        max_u = std::max<int>(max_u, (int)merged.size());
        for (int i = 0; i < c; ++i) {
            const int row = row0 + i;
            size_t k = 0;
            for (int64_t q = A->rp[row]; q < A->rp[row + 1]; ++q) {
                while (merged[k] < A->ci[q]) ++k;
                u_pos[(ubase + k) * cmax + i] = (uint16_t)(q - A->rp[row0]);
            }
        }
        u_off.push_back((int64_t)u_cols.size());
        // j list
        merged.assign(C->ci.begin() + C->rp[row0], C->ci.begin() + C->rp[r]);
        std::sort(merged.begin(), merged.end());
        merged.erase(std::unique(merged.begin(), merged.end()), merged.end());
        const size_t jbase = j_cols.size();
        j_cols.insert(j_cols.end(), merged.begin(), merged.end());
        j_pos.resize(j_cols.size() * cmax, 0xFFFF);
        for (int i = 0; i < c; ++i) {
            const int row = row0 + i;
            size_t k = 0;
            for (int64_t q = C->rp[row]; q < C->rp[row + 1]; ++q) {
                while (merged[k] < C->ci[q]) ++k;
                if (q - C->rp[row] >= 0xFFFF) CHESS_THROW(CHESS_E_UNSUPPORTED, "output row too long");
                j_pos[(jbase + k) * cmax + i] = (uint16_t)(q - C->rp[row]);
            }
        }
        j_off.push_back((int64_t)j_cols.size());
    }
    tile_row0.push_back(A->nb);
    if (Bt->nnzb >= ((int64_t)1 << 31)) CHESS_THROW(CHESS_E_UNSUPPORTED, "Bt pattern has 2^31 or more blocks");
    std::vector<int32_t> j_rec(j_cols.size() * 4);
    for (size_t x = 0; x < j_cols.size(); ++x) {
        const int j = j_cols[x];
        j_rec[4 * x] = j;
        j_rec[4 * x + 1] = (int32_t)Bt->rp[j];
        j_rec[4 * x + 2] = (int32_t)(Bt->rp[j + 1] - Bt->rp[j]);
        j_rec[4 * x + 3] = 0;
    }
    if (max_u >= 32767) CHESS_THROW(CHESS_E_UNSUPPORTED, "row tile with %d distinct columns", max_u);
    int hl = 1;
    while ((1 << hl) < 2 * max_u) ++hl;
    hipStream_t st = ctx->stream;
    upload(P->d_tile_row0, tile_row0, st);
    upload(P->d_u_off, u_off, st);
    upload(P->d_u_cols, u_cols, st);
    upload(P->d_u_pos, u_pos, st);
    upload(P->d_j_off, j_off, st);
    upload(P->d_j_cols, j_cols, st);
    upload(P->d_j_pos, j_pos, st);
    upload(P->d_j_rec, j_rec, st);
    HIPCHECK(hipStreamSynchronize(st));
    P->tile_row0 = tile_row0;
    ProductPlanDev &d = P->dev;
    d.ntiles = (int)tile_row0.size() - 1;
    d.cmax = cmax;
    d.hcap_log2 = hl;
    d.lds_ablocks = lds_ablocks;
    d.max_u = max_u;
    d.max_bt_row = Bt->max_row;
    d.tile_row0 = P->d_tile_row0.as<int32_t>();
    d.u_off = P->d_u_off.as<int64_t>();
    d.u_cols = P->d_u_cols.as<int32_t>();
    d.u_pos = P->d_u_pos.as<uint16_t>();
    d.j_off = P->d_j_off.as<int64_t>();
    d.j_cols = P->d_j_cols.as<int32_t>();
    d.j_pos = P->d_j_pos.as<uint16_t>();
    d.j_rec = P->d_j_rec.as<int32_t>();
    // stage Bt rows in LDS when it fits next to the A tile
    d.stage_bt = (b == 4 && Bt->max_row <= 128) ? 1 : 0;
    if (masked_product_lds_bytes(dtype, b, d) > 160 * 1024) d.stage_bt = 0;
    const size_t lds = masked_product_lds_bytes(dtype, b, d);
    if (lds > 160 * 1024) CHESS_THROW(CHESS_E_UNSUPPORTED, "product tile needs %zu bytes of LDS", lds);
    ctx->plans.push_back(std::move(P));
    return ctx->plans.back().get();
}

// Output-stationary groups of a listed plan (kernels_stat.hip; b = 4): per
// tile, the output blocks in column order (columns by their largest hit count,
// descending) cut into groups of G = 16 (float32 storage) or 4 (float64); a
// group runs R rounds, its largest hit count rounded up to 8; each slot's
// list holds its hits (position in A row i, position in Bt row j) in the
// order of l, then the row's zero block.  Leaves the plan without groups when
// a row is too long for one-byte positions or the packed fields overflow.
static void build_stat_groups(chess_ctx *ctx, ListedPlan *P) {
    const Pattern *A = P->a, *Bt = P->bt, *C = P->c;
    if (A->b != 4 || A->max_row > 254 || Bt->max_row > 255 || Bt->nnzb >= ((int64_t)1 << 22) ||
        C->nnzb >= ((int64_t)1 << 32) - 1)
        return;
    const int G = P->dtype == 0 ? 4 : 16;
    const std::vector<int32_t> &tr0 = P->tile_row0;
    const int ntiles = (int)tr0.size() - 1;
    struct TileOut {
        std::vector<int32_t> ginfo;   // 2 per group (list offset relative to the tile)
        std::vector<uint32_t> slot;   // 2 per slot
        std::vector<uint16_t> list;   // entries, 8 per 16-byte unit
        int ablocks = 0;
        bool overflow = false;
    };
    std::vector<TileOut> outs(ntiles);
    auto work = [&](int t0, int t1) {
        std::vector<uint16_t> ent;
        struct Out { uint32_t blk; int row; int64_t first; int n; int32_t j; };
        std::vector<Out> o;
        for (int t = t0; t < t1; ++t) {
            TileOut &to = outs[t];
            const int row0 = tr0[t], c = tr0[t + 1] - row0;
            int ab[4] = {0, 0, 0, 0}, len[4] = {0, 0, 0, 0};
            int acc = 0;
            for (int r = 0; r < c; ++r) {
                len[r] = (int)(A->rp[row0 + r + 1] - A->rp[row0 + r]);
                ab[r] = acc;
                acc += len[r] + 1;
            }
            to.ablocks = acc;
            if (acc >= 1024 || c > 4) {
                to.overflow = true;
                continue;
            }
            ent.clear();
            o.clear();
            for (int r = 0; r < c; ++r) {
                const int i = row0 + r;
                for (int64_t q = C->rp[i]; q < C->rp[i + 1]; ++q) {
                    const int j = C->ci[q];
                    const int64_t first = (int64_t)ent.size();
                    int64_t pa = A->rp[i], pe = A->rp[i + 1], pb = Bt->rp[j], be = Bt->rp[j + 1];
                    while (pa < pe && pb < be) {
                        const int ca = A->ci[pa], cb = Bt->ci[pb];
                        if (ca < cb) {
                            ++pa;
                        } else if (cb < ca) {
                            ++pb;
                        } else {
                            ent.push_back((uint16_t)((pa - A->rp[i]) | ((pb - Bt->rp[j]) << 8)));
                            ++pa;
                            ++pb;
                        }
                    }
                    o.push_back({(uint32_t)q, r, first, (int)((int64_t)ent.size() - first), j});
                }
            }
            // column order: the outputs of one column j read the same row j of
            // Bt, so a group that holds few columns finds their blocks in L1;
            // columns sorted by their largest hit count keep the counts inside
            // a group close (little padding)
            std::vector<int32_t> jj;
            for (const Out &x : o) jj.push_back(x.j);
            std::sort(jj.begin(), jj.end());
            jj.erase(std::unique(jj.begin(), jj.end()), jj.end());
            std::vector<int> cmax(jj.size(), 0);
            for (const Out &x : o) {
                const size_t k = (size_t)(std::lower_bound(jj.begin(), jj.end(), x.j) - jj.begin());
                cmax[k] = std::max(cmax[k], x.n);
            }
            auto colkey = [&](const Out &x) {
                return cmax[(size_t)(std::lower_bound(jj.begin(), jj.end(), x.j) - jj.begin())];
            };
            std::stable_sort(o.begin(), o.end(), [&](const Out &x, const Out &y) {
                const int kx = colkey(x), ky = colkey(y);
                if (kx != ky) return kx > ky;
                if (x.j != y.j) return x.j < y.j;
                return x.row < y.row;
            });
            // outputs with no hit add nothing (their blocks are written as 0 by
            // a group of their own at the end)
            std::stable_partition(o.begin(), o.end(), [](const Out &x) { return x.n > 0; });
            int64_t list_units = 0;
            for (size_t g0 = 0; g0 < o.size(); g0 += G) {
                const size_t g1 = std::min(o.size(), g0 + (size_t)G);
                // rounds: the group's largest hit count, rounded up to 8
                int nmax = 0;
                for (size_t k = g0; k < g1; ++k) nmax = std::max(nmax, o[k].n);
                const int R = std::max(8, (nmax + 7) & ~7);
                if (R > 0xFFFF) to.overflow = true;
                uint32_t dmask = 0;
                for (size_t k = g0; k < g1; ++k)
                    if (o[k].j == row0 + o[k].row) dmask |= 1u << (k - g0);
                to.ginfo.push_back((int32_t)list_units);
                to.ginfo.push_back((int32_t)(R | (dmask << 16)));
                for (int sl = 0; sl < G; ++sl) {
                    const size_t k = g0 + sl;
                    const bool have = k < g1;
                    const int r = have ? o[k].row : 0;
                    const uint32_t bstart = have ? (uint32_t)Bt->rp[o[k].j] : 0u;
                    to.slot.push_back(have ? o[k].blk : 0xFFFFFFFFu);
                    to.slot.push_back(bstart | ((uint32_t)ab[r] << 22));
                    const uint16_t pad = (uint16_t)len[r];  // the row's zero block, Bt position 0
                    for (int x = 0; x < R; ++x)
                        to.list.push_back(have && x < o[k].n ? ent[(size_t)o[k].first + x] : pad);
                }
                list_units += (int64_t)G * R / 8;
            }
        }
    };
    const int nthr = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    const int chunk = (ntiles + nthr - 1) / nthr;
    for (int k = 0; k < nthr; ++k) {
        const int t0 = k * chunk, t1 = std::min(ntiles, t0 + chunk);
        if (t0 < t1) pool.emplace_back(work, t0, t1);
    }
    for (auto &th : pool) th.join();
    std::vector<int32_t> goff(ntiles + 1, 0);
    int64_t ngroups = 0, nunits = 0;
    int ablocks = 0;
    for (int t = 0; t < ntiles; ++t) {
        if (outs[t].overflow) return;
        goff[t] = (int32_t)ngroups;
        ngroups += (int64_t)outs[t].ginfo.size() / 2;
        nunits += (int64_t)outs[t].list.size() / 8;
        ablocks = std::max(ablocks, outs[t].ablocks);
    }
    goff[ntiles] = (int32_t)ngroups;
    // byte offsets of the lists are 32-bit buffer offsets
    if (ngroups >= ((int64_t)1 << 31) || (nunits + 2) * 16 >= ((int64_t)1 << 31)) return;
    std::vector<int32_t> ginfo((size_t)ngroups * 2);
    std::vector<uint32_t> slot((size_t)ngroups * G * 2);
    std::vector<uint16_t> list((size_t)nunits * 8);
    int64_t gbase = 0, ubase = 0;
    for (int t = 0; t < ntiles; ++t) {
        TileOut &to = outs[t];
        const int64_t ng = (int64_t)to.ginfo.size() / 2;
        for (int64_t g = 0; g < ng; ++g) {
            ginfo[(size_t)(gbase + g) * 2] = (int32_t)(to.ginfo[(size_t)g * 2] + ubase);
            ginfo[(size_t)(gbase + g) * 2 + 1] = to.ginfo[(size_t)g * 2 + 1];
        }
        std::copy(to.slot.begin(), to.slot.end(), slot.begin() + (size_t)gbase * G * 2);
        std::copy(to.list.begin(), to.list.end(), list.begin() + (size_t)ubase * 8);
        gbase += ng;
        ubase += (int64_t)to.list.size() / 8;
        std::vector<int32_t>().swap(to.ginfo);
        std::vector<uint32_t>().swap(to.slot);
        std::vector<uint16_t>().swap(to.list);
    }
    hipStream_t st = ctx->stream;
    upload(P->d_st_goff, goff, st);
    upload(P->d_st_ginfo, ginfo, st);
    upload(P->d_st_slot, slot, st);
    upload(P->d_st_list, list, st);
    HIPCHECK(hipStreamSynchronize(st));
    ListedPlanDev &d = P->dev;
    d.st_goff = P->d_st_goff.as<int32_t>();
    d.st_ginfo = P->d_st_ginfo.as<int32_t>();
    d.st_slot = P->d_st_slot.as<uint32_t>();
    d.st_list = P->d_st_list.p;
    d.st_g = G;
    d.st_ablocks = ablocks;
}

// Symbolic plan with hit lists for C = P_C o (A Bt^T) (see kernels.h,
// ListedPlanDev).  The intersections of sorted rows are computed once here, in
// parallel over tiles.  Returns a plan with usable = false when a row is too
// long for the list format; callers then use the searching kernel.
static ListedPlan *get_listed_plan(chess_ctx *ctx, const Pattern *A, const Pattern *Bt,
                                   const Pattern *C, int dtype,
                                   const std::vector<int32_t> &breaks = {}, int rows = 0) {
    const int cmax = rows > 0 ? rows : pick_cmax(dtype, A->b);
    for (auto &e : ctx->lplans)
        if (e->a == A && e->bt == Bt && e->c == C && e->dtype == dtype && e->breaks == breaks && e->cmax == cmax)
            return e.get();
    auto P = std::make_unique<ListedPlan>();
    P->a = A;
    P->bt = Bt;
    P->c = C;
    P->dtype = dtype;
    P->cmax = cmax;
    P->breaks = breaks;
    std::vector<char> is_break((size_t)A->nb + 1, 0);
    for (int32_t r : breaks)
        if (r >= 0 && r <= A->nb) is_break[r] = 1;
    const int b = A->b;
    const int ew = (A->max_row <= 255 && Bt->max_row <= 255) ? 1 : 2;
    const int max_col_entries = ew == 1 ? 512 : 256;  // LDS list area of a wave: 1 KB
    if (A->max_row > 65535 || Bt->max_row > 65535 || (b == 4 && Bt->max_row > 128) ||
        Bt->nnzb >= ((int64_t)1 << 31)) {
        ctx->lplans.push_back(std::move(P));
        return ctx->lplans.back().get();
    }
    const size_t block_bytes = (size_t)b * b * (dtype == 1 ? 4 : 8);
    // A tile budget: room for CMAX rows of the longest row when that fits
    // (float32 up to 96 KB, float64 up to 80 KB), so tiles are rarely short
    const size_t a_cap = dtype == 1 ? 98304 : 81920;
    const size_t a_budget = std::max<size_t>(dtype == 1 ? 49152 : 40960,
                                             std::min<size_t>(a_cap, (size_t)cmax * A->max_row * block_bytes));
    const int budget_blocks = std::max<int>((int)(a_budget / block_bytes), A->max_row);
    std::vector<int32_t> tile_row0;
    int lds_ablocks = 0;
    for (int r = 0; r < A->nb;) {
        const int row0 = r;
        int64_t blocks = 0;
        while (r < A->nb && r - row0 < cmax) {
            const int64_t len = A->rp[r + 1] - A->rp[r];
            if (r > row0 && (blocks + len > budget_blocks || is_break[r])) break;
            blocks += len;
            ++r;
        }
        tile_row0.push_back(row0);
        lds_ablocks = std::max<int>(lds_ablocks, (int)blocks);
    }
    const int ntiles = (int)tile_row0.size();
    tile_row0.push_back(A->nb);
    P->tile_row0 = tile_row0;
    // hit lists with free slot assignment (float32, b = 4, one-byte positions;
    // Bt rows of at most 128 blocks, so position 255 is outside every row)
    const bool want_lean = dtype == 1 && b == 4 && cmax == 4 && ew == 1;
    struct TileOut {
        std::vector<int32_t> rec;      // 8 per column; entry offsets relative to the tile
        std::vector<uint16_t> ent;     // entry_width 1
        std::vector<uint32_t> ent32;   // entry_width 2
        std::vector<int32_t> lrec;     // free slot assignment: 8 per column, rounds relative to the tile
        std::vector<uint8_t> lent;     // 32 bytes per round
        bool overflow = false;
    };
    std::vector<TileOut> outs(ntiles);
    auto work = [&](int t0, int t1) {
        std::vector<int32_t> cols;
        std::vector<uint16_t> hits[4];
        for (int t = t0; t < t1; ++t) {
            TileOut &o = outs[t];
            const int row0 = tile_row0[t], c = tile_row0[t + 1] - row0;
            cols.assign(C->ci.begin() + C->rp[row0], C->ci.begin() + C->rp[row0 + c]);
            std::sort(cols.begin(), cols.end());
            cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
            for (int j : cols) {
                const int64_t first = ew == 1 ? (int64_t)o.ent.size() : (int64_t)o.ent32.size();
                int32_t counts = 0;
                uint32_t pos01 = 0xFFFFFFFFu, pos23 = 0xFFFFFFFFu;
                int total = 0;
                for (auto &h : hits) h.clear();
                for (int i = 0; i < c; ++i) {
                    const int row = row0 + i;
                    const int64_t q = C->find(row, j);
                    if (q < 0) continue;
                    const uint32_t op = (uint32_t)(q - C->rp[row]);
                    if (i < 2)
                        pos01 = (pos01 & ~(0xFFFFu << (16 * i))) | (op << (16 * i));
                    else
                        pos23 = (pos23 & ~(0xFFFFu << (16 * (i - 2)))) | (op << (16 * (i - 2)));
                    // sorted intersection of A row `row` with Bt row j
                    int64_t pa = A->rp[row], pe = A->rp[row + 1];
                    int64_t pb = Bt->rp[j], be = Bt->rp[j + 1];
                    int n = 0;
                    while (pa < pe && pb < be) {
                        const int ca = A->ci[pa], cb = Bt->ci[pb];
                        if (ca < cb) {
                            ++pa;
                        } else if (cb < ca) {
                            ++pb;
                        } else {
                            const uint32_t ra = (uint32_t)(pa - A->rp[row]);
                            const uint32_t rbt = (uint32_t)(pb - Bt->rp[j]);
                            if (ew == 1) {
                                o.ent.push_back((uint16_t)(ra | (rbt << 8)));
                                if (want_lean) hits[i].push_back((uint16_t)(ra | (rbt << 8)));
                            } else
                                o.ent32.push_back(ra | (rbt << 16));
                            ++n;
                            ++pa;
                            ++pb;
                        }
                    }
                    if (n > 255) o.overflow = true;
                    counts |= (n & 0xFF) << (8 * i);
                    total += n;
                }
                if (total > max_col_entries) o.overflow = true;
                // keep every column's entries 4-byte aligned
                if (ew == 1 && (o.ent.size() & 1)) o.ent.push_back(0);
                o.rec.insert(o.rec.end(), {j, (int32_t)Bt->rp[j], (int32_t)(Bt->rp[j + 1] - Bt->rp[j]),
                                           (int32_t)first, counts, (int32_t)pos01, (int32_t)pos23, 0});
                if (want_lean) {
                    // fewest rounds R with sum_i ceil(cnt_i / R) <= 16 slots; row i
                    // gets n_i = ceil(cnt_i / R) consecutive slots, slot k of the
                    // row takes hits k, k + n_i, ...; R is padded to an even count
                    int R = 0, n[4] = {0, 0, 0, 0};
                    if (total > 0) {
                        for (R = (total + 15) / 16;; ++R) {
                            int need = 0;
                            for (int i = 0; i < 4; ++i) need += ((int)hits[i].size() + R - 1) / R;
                            if (need <= 16) break;
                        }
                        for (int i = 0; i < 4; ++i) n[i] = ((int)hits[i].size() + R - 1) / R;
                        R = (R + 1) & ~1;
                    }
                    const int64_t lfirst = (int64_t)o.lent.size() / 32;
                    const size_t base = o.lent.size();
                    o.lent.resize(base + (size_t)R * 32);
                    for (int r = 0; r < R; ++r) {
                        uint8_t *pa = &o.lent[base + (size_t)r * 32], *pb = pa + 16;
                        for (int sl = 0; sl < 16; ++sl) {
                            pa[sl] = 0;
                            pb[sl] = 255;  // past the list: A's first block times zeros
                        }
                        int s0 = 0;
                        for (int i = 0; i < 4; ++i) {
                            for (int k = 0; k < n[i]; ++k) {
                                const size_t h = (size_t)k + (size_t)n[i] * r;
                                if (h < hits[i].size()) {
                                    pa[s0 + k] = (uint8_t)(hits[i][h] & 0xFF);
                                    pb[s0 + k] = (uint8_t)(hits[i][h] >> 8);
                                }
                            }
                            s0 += n[i];
                        }
                    }
                    if (R > 32) o.overflow = true;  // not reached: at most 4 x 128 hits
                    o.lrec.insert(o.lrec.end(), {j, (int32_t)Bt->rp[j], (int32_t)(Bt->rp[j + 1] - Bt->rp[j]),
                                                 (int32_t)lfirst,
                                                 R | (n[0] << 8) | (n[1] << 13) | (n[2] << 18) | (n[3] << 23),
                                                 (int32_t)pos01, (int32_t)pos23, 0});
                }
            }
        }
    };
    const int nthr = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    const int chunk = (ntiles + nthr - 1) / nthr;
    for (int k = 0; k < nthr; ++k) {
        const int t0 = k * chunk, t1 = std::min(ntiles, t0 + chunk);
        if (t0 < t1) pool.emplace_back(work, t0, t1);
    }
    for (auto &th : pool) th.join();
    std::vector<int64_t> j_off(ntiles + 1, 0);
    int64_t tot_ent = 0, tot_col = 0, tot_rounds = 0;
    for (int t = 0; t < ntiles; ++t) {
        if (outs[t].overflow) {
            ctx->lplans.push_back(std::move(P));
            return ctx->lplans.back().get();
        }
        j_off[t + 1] = j_off[t] + (int64_t)outs[t].rec.size() / 8;
        tot_col += (int64_t)outs[t].rec.size() / 8;
        tot_ent += ew == 1 ? (int64_t)outs[t].ent.size() : (int64_t)outs[t].ent32.size();
        tot_rounds += (int64_t)outs[t].lent.size() / 32;
    }
    // the free-slot kernel addresses hit lists and float64 sums with 31-bit
    // byte offsets
    const bool lean = want_lean && tot_rounds * 32 + 1024 < ((int64_t)1 << 31) &&
                      C->nnzb * 16 * 8 < ((int64_t)1 << 31);
    if (tot_ent >= ((int64_t)1 << 31)) {
        ctx->lplans.push_back(std::move(P));
        return ctx->lplans.back().get();
    }
    std::vector<int32_t> rec((size_t)tot_col * 8);
    std::vector<uint16_t> ent;
    std::vector<uint32_t> ent32;
    if (ew == 1) ent.resize((size_t)tot_ent); else ent32.resize((size_t)tot_ent);
    std::vector<int32_t> lrec(lean ? (size_t)tot_col * 8 : 0);
    // padded so that the last column's 4-word-per-lane prefetch stays inside
    std::vector<uint8_t> lent(lean ? (size_t)tot_rounds * 32 + 1024 : 0, 0);
    int64_t ebase = 0, lbase = 0;
    for (int t = 0; t < ntiles; ++t) {
        TileOut &o = outs[t];
        const size_t nrec = o.rec.size() / 8;
        for (size_t x = 0; x < nrec; ++x) {
            int32_t *r = &rec[(size_t)(j_off[t] + x) * 8];
            std::copy(o.rec.begin() + 8 * x, o.rec.begin() + 8 * x + 8, r);
            r[3] = (int32_t)(r[3] + ebase);
            if (lean) {
                int32_t *lr = &lrec[(size_t)(j_off[t] + x) * 8];
                std::copy(o.lrec.begin() + 8 * x, o.lrec.begin() + 8 * x + 8, lr);
                lr[3] = (int32_t)(lr[3] + lbase);
            }
        }
        if (lean) {
            std::copy(o.lent.begin(), o.lent.end(), lent.begin() + lbase * 32);
            lbase += (int64_t)o.lent.size() / 32;
        }
        std::vector<int32_t>().swap(o.lrec);
        std::vector<uint8_t>().swap(o.lent);
        if (ew == 1) {
            std::copy(o.ent.begin(), o.ent.end(), ent.begin() + ebase);
            ebase += (int64_t)o.ent.size();
        } else {
            std::copy(o.ent32.begin(), o.ent32.end(), ent32.begin() + ebase);
            ebase += (int64_t)o.ent32.size();
        }
        std::vector<int32_t>().swap(o.rec);
        std::vector<uint16_t>().swap(o.ent);
        std::vector<uint32_t>().swap(o.ent32);
    }
    // pad so that the last column's 4-word prefetch stays inside the buffer
    if (ew == 1) ent.resize(ent.size() + 1024, 0); else ent32.resize(ent32.size() + 512, 0);
    hipStream_t st = ctx->stream;
    upload(P->d_tile_row0, tile_row0, st);
    upload(P->d_j_off, j_off, st);
    upload(P->d_j_rec, rec, st);
    if (ew == 1) upload(P->d_entries, ent, st); else upload(P->d_entries, ent32, st);
    if (lean) {
        upload(P->d_lean_rec, lrec, st);
        upload(P->d_lean_ent, lent, st);
    }
    HIPCHECK(hipStreamSynchronize(st));
    ListedPlanDev &d = P->dev;
    d.ntiles = ntiles;
    d.cmax = cmax;
    d.lds_ablocks = lds_ablocks;
    d.max_bt_row = Bt->max_row;
    d.max_entries = max_col_entries;
    d.entry_width = ew;
    d.tile_row0 = P->d_tile_row0.as<int32_t>();
    d.j_off = P->d_j_off.as<int64_t>();
    d.j_rec = P->d_j_rec.as<int32_t>();
    d.entries = P->d_entries.p;
    if (lean) {
        d.lean_rec = P->d_lean_rec.as<int32_t>();
        d.lean_ent = P->d_lean_ent.as<uint8_t>();
    }
    for (int t = 0; t < ntiles; ++t) d.max_cols = std::max<int>(d.max_cols, (int)(j_off[t + 1] - j_off[t]));
    d.off31 = C->nnzb * b * b * 8 < ((int64_t)1 << 31) && (tot_ent + 1024) * 2 * ew < ((int64_t)1 << 31);
    if (b == 4 && d.off31) build_stat_groups(ctx, P.get());
    P->usable = listed_product_lds_bytes(dtype, b, d) <= 160 * 1024;
    ctx->lplans.push_back(std::move(P));
    return ctx->lplans.back().get();
}

// The product launchers keep, per kernel, a process-wide record of the
// dynamic LDS limit they have raised (hipFuncSetAttribute); this lock keeps
// that record consistent when contexts launch from several threads at once.
static std::mutex g_launch_mu;

static hipError_t launch_listed_locked(int dtype, int b, const ListedPlanDev &d, const ProductOperands &ops,
                                       const Epilogue &ep, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_launch_mu);
    return launch_listed_product(dtype, b, d, ops, ep, st);
}

// C = P_C o (A Bt^T) with an epilogue.  A, Bt, C value arrays in dtype.
static void product(chess_ctx *ctx, int dtype, const ProductPlan *plan, const void *a,
                    const void *bt, void *c, const Epilogue &ep) {
    ProductOperands ops;
    ops.a_rp = plan->a->d_rp.as<int64_t>();
    ops.a_val = a;
    ops.bt_rp = plan->bt->d_rp.as<int64_t>();
    ops.bt_ci = plan->bt->d_ci.as<int32_t>();
    ops.bt_val = bt;
    ops.c_rp = plan->c->d_rp.as<int64_t>();
    ops.c_out = c;
    std::lock_guard<std::mutex> lk(g_launch_mu);
    HIPCHECK(launch_masked_product(dtype, plan->a->b, plan->dev, ops, ep, ctx->stream));
}

static void product_listed(chess_ctx *ctx, int dtype, const ListedPlan *plan, const void *a,
                           const void *bt, void *c, const Epilogue &ep, int opmode = 0,
                           const void *bt_hi = nullptr, const void *bt_lo = nullptr) {
    ProductOperands ops;
    ops.opmode = opmode;
    ops.bt_hi = bt_hi;
    ops.bt_lo = bt_lo;
    ops.a_rp = plan->a->d_rp.as<int64_t>();
    ops.a_val = a;
    ops.bt_rp = plan->bt->d_rp.as<int64_t>();
    ops.bt_ci = plan->bt->d_ci.as<int32_t>();
    ops.bt_val = bt;
    ops.c_rp = plan->c->d_rp.as<int64_t>();
    ops.c_out = c;
    HIPCHECK(launch_listed_locked(dtype, plan->a->b, plan->dev, ops, ep, ctx->stream));
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

static size_t vbytes(const Pattern *P, int dtype) {
    return (size_t)P->nnzb * P->b * P->b * (dtype == 1 ? 4 : 8);
}

static double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t st;
    explicit Timer(hipStream_t s) : st(s) {
        HIPCHECK(hipEventCreate(&a));
        HIPCHECK(hipEventCreate(&b));
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    void start() { HIPCHECK(hipEventRecord(a, st)); }
    double stop() {
        HIPCHECK(hipEventRecord(b, st));
        HIPCHECK(hipEventSynchronize(b));
        float ms = 0;
        HIPCHECK(hipEventElapsedTime(&ms, a, b));
        return ms;
    }
};

// Gershgorin bounds of a float64 matrix on pattern P.
static void gershgorin(chess_ctx *ctx, const Pattern *P, const double *val, double *lo, double *hi) {
    const int nparts = 256;
    DevBuf part(sizeof(double) * (2 * nparts + 2));
    double *plo = part.as<double>(), *phi = plo + nparts, *out = phi + nparts;
    HIPCHECK(launch_gershgorin(P->b, P->nb, P->d_rp.as<int64_t>(), P->d_ci.as<int32_t>(), val, plo, phi, nparts, ctx->stream));
    HIPCHECK(launch_minmax(nparts, plo, phi, out, ctx->stream));
    double h[2];
    HIPCHECK(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(hipStreamSynchronize(ctx->stream));
    *lo = h[0];
    *hi = h[1];
}

// k steps of Lanczos with full reorthogonalisation on a float64 matrix;
// returns the extreme Ritz values and their residual norms.
static void lanczos(chess_ctx *ctx, const Pattern *P, const double *val, int k, double *tmin,
                    double *tmax, double *rmin, double *rmax) {
    const int64_t n = P->n();
    k = (int)std::min<int64_t>(k, n);
    hipStream_t st = ctx->stream;
    DevBuf V(sizeof(double) * (size_t)(k + 1) * n), w(sizeof(double) * n);
    const int nparts = 128;
    DevBuf part(sizeof(double) * (size_t)(k + 1) * nparts), h(sizeof(double) * (k + 2));
    // seeded start vector (xorshift64*, normalised on the device)
    std::vector<double> v0(n);
    uint64_t s = 0x9E3779B97F4A7C15ull;
    for (int64_t i = 0; i < n; ++i) {
        s ^= s >> 12;
        s ^= s << 25;
        s ^= s >> 27;
        v0[i] = (double)((s * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    }
    HIPCHECK(hipMemcpyAsync(w.p, v0.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
    double *Vd = V.as<double>(), *wd = w.as<double>(), *hd = h.as<double>(), *pd = part.as<double>();
    HIPCHECK(launch_multidot(1, n, wd, wd, pd, nparts, st));
    HIPCHECK(launch_reduce_rows(1, nparts, pd, hd + k + 1, st));
    HIPCHECK(launch_normalize(n, wd, hd + k + 1, Vd, st));
    std::vector<double> alpha, beta;
    double beta_last = 0.0;
    for (int j = 0; j < k; ++j) {
        double *vj = Vd + (size_t)j * n;
        HIPCHECK(launch_spmv(P->b, P->nb, P->d_rp.as<int64_t>(), P->d_ci.as<int32_t>(), val, vj, wd, st));
        for (int pass = 0; pass < 2; ++pass) {
            HIPCHECK(launch_multidot(j + 1, n, Vd, wd, pd, nparts, st));
            HIPCHECK(launch_reduce_rows(j + 1, nparts, pd, hd, st));
            if (pass == 0) {
                double aj;
                HIPCHECK(hipMemcpyAsync(&aj, hd + j, sizeof(double), hipMemcpyDeviceToHost, st));
                HIPCHECK(hipStreamSynchronize(st));
                alpha.push_back(aj);
            }
            HIPCHECK(launch_multiaxpy(j + 1, n, Vd, hd, wd, st));
        }
        HIPCHECK(launch_multidot(1, n, wd, wd, pd, nparts, st));
        HIPCHECK(launch_reduce_rows(1, nparts, pd, hd + k + 1, st));
        double nrm2;
        HIPCHECK(hipMemcpyAsync(&nrm2, hd + k + 1, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        const double bj = std::sqrt(std::max(nrm2, 0.0));
        beta_last = bj;
        if (j + 1 == k || bj < 1e-12) break;
        beta.push_back(bj);
        HIPCHECK(launch_normalize(n, wd, hd + k + 1, Vd + (size_t)(j + 1) * n, st));
    }
    beta.resize(alpha.size() > 0 ? alpha.size() - 1 : 0);
    hostmath::tridiag_extremes(alpha, beta, beta_last, tmin, tmax, rmin, rmax);
}

// ---------------------------------------------------------------------------
// the Chebyshev chain
// ---------------------------------------------------------------------------

struct ChainRequest {
    const Pattern *PM = nullptr;  // pattern of M~
    const double *Mt = nullptr;   // M~ (float64) on PM
    const Pattern *PK = nullptr;  // pattern of the T_k
    int n_pl = 0;
    int nq = 0;
    const double *coef = nullptr;  // host [nq][n_pl]
    double *acc[4] = {nullptr, nullptr, nullptr, nullptr};  // device, float64 on PK (transposed storage)
    int dtype = 0;
    int opmode = 0;        // operand mode of the products (bfloat16 forms: float32 storage)
    void *hist = nullptr;  // optional device [n_pl][nnzK*b*b] in dtype
    std::vector<double> *moments = nullptr;
    const char *label = "chain";  // stage name given to the progress callback
    double kernel_ms = 0.0;  // out: device time of the product launches
    int variant = -1;        // out: kernel variant of the listed product (-1: searching kernel)
    int tile_rows = 0;       // out: rows per tile of the listed product's plan
    int products = 0;        // out: product launches of the chain
};

// Kernel variant of a listed plan.  CHESS_LISTED_VARIANT=<v> in the
// environment forces variant v; otherwise the first chain long enough to pay
// for it times every variant on its own operands (one warm-up and three timed
// launches each, written to a scratch output) and the fastest one is kept for
// the plan's lifetime.
// Chooses the kernel variant of a chain pass by timing them on its first
// product; passes with float64 sums (nacc > 0, acc = the pass's sums, left
// unchanged: the timed launches add them with weight 0) are timed apart
// from passes without.
static void select_listed_variant(chess_ctx *ctx, ListedPlan *lp, int dtype, int n_pl,
                                  const void *a, const void *bt, const void *prev, int opmode = 0,
                                  const void *bt_hi = nullptr, const void *bt_lo = nullptr,
                                  int nacc = 0, double *const *acc = nullptr) {
    const int pass = nacc > 0 ? 1 : 0;
    const int b = lp->a->b;
    const int nvar = listed_product_variants(dtype, b, lp->dev);
    if (const char *env = std::getenv("CHESS_LISTED_VARIANT")) {
        char *end = nullptr;
        const long v = std::strtol(env, &end, 10);
        if (end == env || !listed_product_variant_ok(dtype, b, lp->dev, (int)v, opmode))
            CHESS_THROW(CHESS_E_ARG, "CHESS_LISTED_VARIANT=%s: no such kernel variant here (ids 0..%d)", env, nvar - 1);
        lp->dev.variant = (int)v;
        if (listed_product_lds_bytes(dtype, b, lp->dev, opmode) > 160 * 1024)
            CHESS_THROW(CHESS_E_UNSUPPORTED, "kernel variant %ld needs more than 160 KB of LDS", v);
        return;
    }
    if (lp->tuned_variant[opmode][pass] >= 0) {
        lp->dev.variant = lp->tuned_variant[opmode][pass];
        return;
    }
    // untimed default: b = 4, the output-stationary kernel (float32 with 8
    // waves, float64 with 16; without its groups, the free-slot kernel or
    // operands from global memory); b = 9 float32, the MFMA kernel with
    // pipelined columns and 8 waves (or without); variant 0 otherwise
    auto fits = [&](int v) {
        ListedPlanDev d = lp->dev;
        d.variant = v;
        return listed_product_variant_ok(dtype, b, d, v, opmode) && listed_product_lds_bytes(dtype, b, d, opmode) <= 160 * 1024;
    };
    if (opmode != 0) {
        if (!fits(kStatVariantF32))
            CHESS_THROW(CHESS_E_UNSUPPORTED, "bfloat16 operands need b = 4 and rows of at most 254 blocks");
        lp->dev.variant = kStatVariantF32;
    } else if (b == 4 && lp->cmax != 4) {
        // tiles of other heights: the output-stationary kernel only
        const int v = dtype == 1 ? kStatVariantF32 : kStatVariantF64 + 2;
        if (!fits(v)) CHESS_THROW(CHESS_E_UNSUPPORTED, "tiles of %d rows need the output-stationary kernel", lp->cmax);
        lp->dev.variant = v;
    } else if (nvar == 1)
        lp->dev.variant = 0;
    else if (b == 4 && dtype == 1)
        lp->dev.variant = fits(kStatVariantF32) ? kStatVariantF32 : fits(20) ? 20 : 8;
    else if (b == 9)
        lp->dev.variant = fits(3) ? 3 : 2;
    else
        lp->dev.variant = fits(kStatVariantF64 + 2) ? kStatVariantF64 + 2 : 2;
    if (nvar == 1 || n_pl < 64) return;  // too short a chain to time variants on
    hipStream_t st = ctx->stream;
    DevBuf out(vbytes(lp->c, dtype));
    ProductOperands ops;
    ops.a_rp = lp->a->d_rp.as<int64_t>();
    ops.a_val = a;
    ops.bt_rp = lp->bt->d_rp.as<int64_t>();
    ops.bt_ci = lp->bt->d_ci.as<int32_t>();
    ops.bt_val = bt;
    ops.c_rp = lp->c->d_rp.as<int64_t>();
    ops.c_out = out.p;
    ops.opmode = opmode;
    ops.bt_hi = bt_hi;
    ops.bt_lo = bt_lo;
    Epilogue ep;
    ep.alpha = 2.0;
    ep.beta = -1.0;
    ep.prev = prev;
    ep.nacc = acc ? nacc : 0;
    for (int q = 0; q < ep.nacc; ++q) {
        ep.acc[q] = acc[q];
        ep.coef[q] = 0.0;
    }
    Timer tm(st);
    double best = 0.0;
    int best_v = -1;
    for (int v = 0; v < nvar; ++v) {
        ListedPlanDev d = lp->dev;
        d.variant = v;
        if (!listed_product_variant_ok(dtype, b, d, v, opmode) || listed_product_lds_bytes(dtype, b, d, opmode) > 160 * 1024) continue;
        HIPCHECK(launch_listed_locked(dtype, b, d, ops, ep, st));
        tm.start();
        for (int r = 0; r < 3; ++r) HIPCHECK(launch_listed_locked(dtype, b, d, ops, ep, st));
        const double ms = tm.stop();
        if (best_v < 0 || ms < best) {
            best = ms;
            best_v = v;
        }
    }
    if (best_v < 0) best_v = lp->dev.variant;
    lp->tuned_variant[opmode][pass] = best_v;
    lp->tuned_ms[opmode][pass] = best_v >= 0 ? best / 3 : -1.0;
    lp->dev.variant = best_v;
}

// Row-tile height of a chain's plan (b = 4): the plan with the default 4-row
// tiles against one with 2-row tiles (twice the workgroups, each row of Bt
// read by twice the tiles; the output-stationary kernel only), each with its
// fastest variant, on the chain's first product; the 2-row plan is kept for
// the pattern and pass type when it is at least 3 % faster (both plans stay
// cached).  CHESS_TILE_ROWS in the environment forces a height.  Returns the
// plan to use (its variant set).
static ListedPlan *tune_tile_rows(chess_ctx *ctx, ListedPlan *lp, int dtype, int n_pl,
                                  const void *a, const void *bt, const void *prev, int opmode,
                                  const void *bt_hi, const void *bt_lo, int nacc, double *const *acc) {
    const Pattern *A = lp->a, *Bt = lp->bt, *C = lp->c;
    auto pick = [&](ListedPlan *p) {
        select_listed_variant(ctx, p, dtype, n_pl, a, bt, prev, opmode, bt_hi, bt_lo, nacc, acc);
        return p;
    };
    auto stat_ready = [&](ListedPlan *p) {
        const int v0 = dtype == 0 ? kStatVariantF64 : kStatVariantF32;
        return p->usable && listed_product_variant_ok(dtype, 4, p->dev, v0, opmode);
    };
    if (A->b != 4) return pick(lp);
    if (const char *env = std::getenv("CHESS_TILE_ROWS")) {
        const int rows = std::atoi(env);
        if (rows != 1 && rows != 2 && rows != 4) CHESS_THROW(CHESS_E_ARG, "CHESS_TILE_ROWS=%s: 1, 2 or 4 rows", env);
        if (rows == lp->cmax) return pick(lp);
        ListedPlan *alt = get_listed_plan(ctx, A, Bt, C, dtype, lp->breaks, rows);
        if (!stat_ready(alt)) CHESS_THROW(CHESS_E_UNSUPPORTED, "CHESS_TILE_ROWS=%d: no output-stationary plan", rows);
        return pick(alt);
    }
    // a variant forced by CHESS_LISTED_VARIANT names a kernel of the default
    // plan (4-row tiles)
    if (std::getenv("CHESS_LISTED_VARIANT")) return pick(lp);
    const int pass = nacc > 0 ? 1 : 0;
    for (const auto &tc : ctx->tile_choices)
        if (tc.a == A && tc.bt == Bt && tc.dtype == dtype && tc.breaks == lp->breaks && tc.opmode == opmode &&
            tc.pass == pass)
            return pick(tc.rows == lp->cmax ? lp : get_listed_plan(ctx, A, Bt, C, dtype, lp->breaks, tc.rows));
    pick(lp);
    const double t4 = lp->tuned_ms[opmode][pass];
    if (n_pl < 64 || t4 <= 0.0 || !stat_ready(lp)) return lp;  // too short to time, or untimed
    ListedPlan *alt = get_listed_plan(ctx, A, Bt, C, dtype, lp->breaks, 2);
    int rows = lp->cmax;
    if (stat_ready(alt)) {
        pick(alt);
        const double t2 = alt->tuned_ms[opmode][pass];
        if (t2 > 0.0 && t2 < 0.97 * t4) rows = 2;
    }
    ctx->tile_choices.push_back({A, Bt, dtype, lp->breaks, opmode, pass, rows});
    return rows != lp->cmax ? alt : pick(lp);
}

// Runs T_0 .. T_{n_pl-1} in transposed storage U_k = T_k^T (see kernels.hip).
static void run_chain(chess_ctx *ctx, ChainRequest &rq) {
    hipStream_t st = ctx->stream;
    const Pattern *PM = rq.PM, *PK = rq.PK;
    const int b = PK->b;
    const int dtype = rq.dtype;
    const int64_t nK = PK->nnzb * b * b;
    const EmbedMap *emb = get_embed(ctx, PM, PK, "M~ in the chain pattern");
    ListedPlan *lplan = get_listed_plan(ctx, PK, PM, PK, dtype);
    const ProductPlan *plan = lplan->usable ? nullptr : get_plan(ctx, PK, PM, PK, dtype);
    const size_t tb = vbytes(PK, dtype);
    // Bt gets 16 KB of slack: the listed kernel reads whole 64-lane rounds of a row
    DevBuf U0(tb), U1(tb), Bt(vbytes(PM, dtype) + 16384);
    // Bt = M~^T on PM (row j of Bt = column j of M~)
    HIPCHECK(launch_scatter_blocks(dtype, b, PM->nnzb, PM->d_tmap.as<int64_t>(), rq.Mt, Bt.p, 1, st));
    // bfloat16 operand forms of Bt (hi, and lo for the three-product split)
    DevBuf Bhi, Blo;
    if (rq.opmode != 0) {
        if (dtype != 1 || !lplan->usable)
            CHESS_THROW(CHESS_E_UNSUPPORTED, "bfloat16 operands need b = 4 and rows of at most 254 blocks");
        const int64_t nv = PM->nnzb * b * b;
        Bhi.alloc(sizeof(uint16_t) * (size_t)nv + 16384);
        if (rq.opmode == kStatBF16X3) Blo.alloc(sizeof(uint16_t) * (size_t)nv + 16384);
        HIPCHECK(launch_split_bf16(nv, Bt.as<float>(), Bhi.as<unsigned short>(),
                                   rq.opmode == kStatBF16X3 ? Blo.as<unsigned short>() : nullptr, st));
    }
    // U_0 = I, U_1 = M~^T placed in PK
    HIPCHECK(launch_fill_identity(dtype, b, PK->nnzb, PK->d_brow.as<int32_t>(), PK->d_ci.as<int32_t>(), U0.p, st));
    HIPCHECK(launch_zero(U1.p, tb, st));
    if (rq.n_pl > 1)
        HIPCHECK(launch_scatter_blocks(dtype, b, PM->nnzb, emb->d_map_t.as<int64_t>(), rq.Mt, U1.p, 1, st));
    if (lplan->usable) {
        lplan = tune_tile_rows(ctx, lplan, dtype, rq.n_pl, U1.p, Bt.p, U0.p, rq.opmode, Bhi.p, Blo.p, rq.nq,
                               rq.acc);
        rq.variant = lplan->dev.variant;
        rq.tile_rows = lplan->cmax;
    }
    for (int q = 0; q < rq.nq; ++q) {
        const double *c = rq.coef + (size_t)q * rq.n_pl;
        HIPCHECK(launch_axpby_to_f64(dtype, nK, 0.5 * c[0], U0.p, rq.n_pl > 1 ? c[1] : 0.0, U1.p, rq.acc[q], st));
    }
    if (rq.hist) {
        HIPCHECK(hipMemcpyAsync(rq.hist, U0.p, tb, hipMemcpyDeviceToDevice, st));
        if (rq.n_pl > 1)
            HIPCHECK(hipMemcpyAsync((char *)rq.hist + tb, U1.p, tb, hipMemcpyDeviceToDevice, st));
    }
    const int ntiles = lplan->usable ? lplan->dev.ntiles : plan->dev.ntiles;
    const int nsteps = std::max(rq.n_pl, 2);
    // Moments-only chains (no sums, no history) run to T_K, K = ceil((n_pl -
    // 1) / 2), and take the rest of the moments from the product rule of
    // Chebyshev polynomials, 2 T_m T_n = T_{m+n} + T_{|m-n|}: t_{2m} =
    // 2 <T_m, T_m> - n and t_{2m+1} = 2 <T_{m+1}, T_m> - t_1, with <., .> the
    // Frobenius product of the stored blocks.  This holds for the truncated
    // chain too: column j of the truncated T_m is T_m(M_j) e_j with M_j the
    // symmetric compression of M~ to that column's support (the columns obey
    // the recursion independently), so e_j^T T_{2m}(M_j) e_j = 2 |T_m e_j|^2 - 1.
    const bool halve = rq.nq == 0 && !rq.hist && rq.moments && rq.n_pl > 4 && !std::getenv("CHESS_FULL_MOMENTS");
    const int last = halve ? rq.n_pl / 2 : rq.n_pl - 1;  // highest T_m computed (ceil((n_pl - 1) / 2))
    // dot-pair workgroups: enough to stream the T_m arrays at full rate
    const int dparts = (int)std::min<int64_t>(2048, std::max<int64_t>(64, nK / 4096));
    DevBuf part(sizeof(double) * (size_t)nsteps * std::max(ntiles, 256));
    // the output-stationary kernel adds the Frobenius products of its output
    // per tile (Epilogue::sq_partial); the other kernels leave them to
    // k_dot_pair after each product
    const int v0s = dtype == 1 ? kStatVariantF32 : kStatVariantF64;
    const bool fused = halve && lplan->usable &&
                       (rq.opmode != 0 || (b == 4 && lplan->dev.variant >= v0s && lplan->dev.variant <= v0s + 2));
    DevBuf dpart, dred, fpart, fred;
    if (halve) {
        dpart.alloc(sizeof(double) * 2 * (size_t)dparts * (fused ? 1 : last));
        dred.alloc(sizeof(double) * 2 * (size_t)last);
        if (fused) {
            fpart.alloc(sizeof(double) * 2 * (size_t)ntiles * last);
            fred.alloc(sizeof(double) * 2 * (size_t)last);
        }
    }
    DevBuf mom(sizeof(double) * nsteps);
    double *pd = part.as<double>();
    const int tparts = 256;
    // moments 0 and 1
    HIPCHECK(launch_trace(dtype, b, PK->nb, PK->d_diag.as<int64_t>(), U0.p, pd, tparts, st));
    HIPCHECK(launch_reduce_rows(1, tparts, pd, mom.as<double>(), st));
    if (rq.n_pl > 1) {
        HIPCHECK(launch_trace(dtype, b, PK->nb, PK->d_diag.as<int64_t>(), U1.p, pd + tparts, tparts, st));
        HIPCHECK(launch_reduce_rows(1, tparts, pd + tparts, mom.as<double>() + 1, st));
    }
    // <T_m, T_m> and <T_m, T_{m-1}> go to block m - 1 of the halving partials
    auto dots = [&](int m, const void *tm, const void *tm1) {
        HIPCHECK(launch_dot_pair(dtype, nK, tm, tm1, dpart.as<double>() + 2 * (size_t)dparts * (m - 1), dparts, st));
    };
    void *ucur = U1.p, *uprev = U0.p;
    Timer tm(st);
    tm.start();
    if (halve) dots(1, U1.p, U0.p);
    rq.products = 0;
    for (int k = 1; k + 1 <= last; ++k) {
        Epilogue ep;
        ep.alpha = 2.0;
        ep.beta = -1.0;
        ep.prev = uprev;
        ep.nacc = rq.nq;
        for (int q = 0; q < rq.nq; ++q) {
            ep.acc[q] = rq.acc[q];
            ep.coef[q] = rq.coef[(size_t)q * rq.n_pl + k + 1];
        }
        ep.hist = rq.hist ? (char *)rq.hist + (size_t)(k + 1) * tb : nullptr;
        ep.trace_partial = halve ? nullptr : pd + (size_t)(k + 1) * ntiles;
        if (fused) {
            // rows m - 1 of the <T_m, T_m> and <T_m, T_{m-1}> partials, m = k + 1
            ep.sq_partial = fpart.as<double>() + (size_t)k * ntiles;
            ep.xy_partial = fpart.as<double>() + (size_t)(last + k) * ntiles;
        }
        if (lplan->usable)
            product_listed(ctx, dtype, lplan, ucur, Bt.p, uprev, ep, rq.opmode, Bhi.p, Blo.p);
        else
            product(ctx, dtype, plan, ucur, Bt.p, uprev, ep);
        rq.products++;
        std::swap(ucur, uprev);
        if (halve && !fused) dots(k + 1, ucur, uprev);
        if (ctx->progress && (k + 1) % ctx->progress_every == 0) {
            HIPCHECK(hipStreamSynchronize(st));
            ctx->progress(ctx->progress_user, rq.label, halve ? 2 * (k + 1) : k + 1, rq.n_pl);
        }
    }
    rq.kernel_ms = tm.stop();
    if (halve) {
        HIPCHECK(launch_reduce_rows(fused ? 2 : 2 * last, dparts, dpart.as<double>(), dred.as<double>(), st));
        std::vector<double> red(2 * (size_t)last);
        HIPCHECK(hipMemcpyAsync(red.data(), dred.p, sizeof(double) * (fused ? 2 : red.size()), hipMemcpyDeviceToHost, st));
        if (fused && last > 1) {
            // rows m = 2 .. last of the per-tile partials
            HIPCHECK(launch_reduce_rows(2 * last, ntiles, fpart.as<double>(), fred.as<double>(), st));
            std::vector<double> f(2 * (size_t)last);
            HIPCHECK(hipMemcpyAsync(f.data(), fred.p, sizeof(double) * f.size(), hipMemcpyDeviceToHost, st));
            HIPCHECK(hipStreamSynchronize(st));
            for (int m = 2; m <= last; ++m) {
                red[2 * (size_t)(m - 1)] = f[(size_t)(m - 1)];
                red[2 * (size_t)(m - 1) + 1] = f[(size_t)(last + m - 1)];
            }
        }
        rq.moments->assign(rq.n_pl, 0.0);
        HIPCHECK(hipMemcpyAsync(rq.moments->data(), mom.p, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        std::vector<double> &t = *rq.moments;
        const double n = (double)PK->n();
        // red[2 (m - 1)] = <T_m, T_m>, red[2 (m - 1) + 1] = <T_m, T_{m-1}>
        for (int j = 2; j < rq.n_pl; ++j) {
            const int m = j / 2;
            t[j] = (j % 2 == 0) ? 2.0 * red[2 * (size_t)(m - 1)] - n : 2.0 * red[2 * (size_t)m + 1] - t[1];
        }
        return;
    }
    if (rq.n_pl > 2)
        HIPCHECK(launch_reduce_rows(rq.n_pl - 2, ntiles, pd + 2 * (size_t)ntiles, mom.as<double>() + 2, st));
    if (rq.moments) {
        rq.moments->assign(rq.n_pl, 0.0);
        HIPCHECK(hipMemcpyAsync(rq.moments->data(), mom.p, sizeof(double) * rq.n_pl, hipMemcpyDeviceToHost, st));
    }
    HIPCHECK(hipStreamSynchronize(st));
}

// Chain over a batch of independent systems laid out block-diagonally: system
// s owns block rows [row0[s], row0[s+1]) of PM and PK.  Row tiles never
// straddle systems, so each tile's accumulator weight is that of its system
// (coef_tab [nq][n_pl][nsys], zero past a system's own degree) and the trace
// partials of a system's tiles sum to its moments (out [n_pl][nsys]).  The
// products of steps 2 .. n_pl-2 are recorded once into a HIP graph and
// launched as one graph.
struct BatchChain {
    const Pattern *PM = nullptr, *PK = nullptr;
    const double *Mt = nullptr;
    int n_pl = 0, nq = 0, dtype = 0;
    int opmode = 0;  // operand mode of the products (bfloat16 forms: float32 storage)
    const double *coef_tab = nullptr;
    double *acc[4] = {nullptr, nullptr, nullptr, nullptr};
    const std::vector<int32_t> *row0 = nullptr;
    const int32_t *d_row_sys = nullptr;
    // each system's own number of terms (n_pl is their maximum): a system's
    // tiles stop once its chain is complete
    const std::vector<int> *sys_npl = nullptr;
    bool use_graph = true;
    std::vector<double> *moments = nullptr;
    double kernel_ms = 0.0;
    int variant = -1;
    int graph_nodes = 0;
};

static void run_chain_batched(chess_ctx *ctx, BatchChain &rq) {
    hipStream_t st = ctx->stream;
    const Pattern *PM = rq.PM, *PK = rq.PK;
    const int b = PK->b, dtype = rq.dtype, n_pl = rq.n_pl;
    const std::vector<int32_t> &row0 = *rq.row0;
    const int nsys = (int)row0.size() - 1;
    const size_t esz = dtype == 1 ? 4 : 8;
    const EmbedMap *emb = get_embed(ctx, PM, PK, "M~ in the chain pattern");
    const std::vector<int32_t> breaks(row0.begin(), row0.end() - 1);
    ListedPlan *lp = get_listed_plan(ctx, PK, PM, PK, dtype, breaks);
    // rows too long for the hit lists: the searching product, on tiles that
    // also start at every system
    const ProductPlan *plan = lp->usable ? nullptr : get_plan(ctx, PK, PM, PK, dtype, breaks);
    if (!lp->usable && rq.opmode != 0)
        CHESS_THROW(CHESS_E_UNSUPPORTED, "bfloat16 operands need b = 4 and rows of at most 254 blocks");
    const size_t tb = vbytes(PK, dtype);
    DevBuf U0(tb), U1(tb), Bt(vbytes(PM, dtype) + 16384);
    HIPCHECK(launch_scatter_blocks(dtype, b, PM->nnzb, PM->d_tmap.as<int64_t>(), rq.Mt, Bt.p, 1, st));
    HIPCHECK(launch_fill_identity(dtype, b, PK->nnzb, PK->d_brow.as<int32_t>(), PK->d_ci.as<int32_t>(), U0.p, st));
    HIPCHECK(launch_zero(U1.p, tb, st));
    HIPCHECK(launch_scatter_blocks(dtype, b, PM->nnzb, emb->d_map_t.as<int64_t>(), rq.Mt, U1.p, 1, st));
    DevBuf Bhi, Blo;
    if (rq.opmode != 0) {
        if (dtype != 1) CHESS_THROW(CHESS_E_UNSUPPORTED, "bfloat16 operands need float32 storage");
        const int64_t nv = PM->nnzb * b * b;
        Bhi.alloc(sizeof(uint16_t) * (size_t)nv + 16384);
        if (rq.opmode == kStatBF16X3) Blo.alloc(sizeof(uint16_t) * (size_t)nv + 16384);
        HIPCHECK(launch_split_bf16(nv, Bt.as<float>(), Bhi.as<unsigned short>(),
                                   rq.opmode == kStatBF16X3 ? Blo.as<unsigned short>() : nullptr, st));
    }
    if (lp->usable) {
        lp = tune_tile_rows(ctx, lp, dtype, n_pl, U1.p, Bt.p, U0.p, rq.opmode, Bhi.p, Blo.p, rq.nq, rq.acc);
        rq.variant = lp->dev.variant;
    } else {
        rq.variant = -1;
    }
    DevBuf dcoef(sizeof(double) * (size_t)std::max(rq.nq, 1) * n_pl * nsys);
    if (rq.nq)
        HIPCHECK(hipMemcpyAsync(dcoef.p, rq.coef_tab, sizeof(double) * (size_t)rq.nq * n_pl * nsys, hipMemcpyHostToDevice, st));
    // sum' starts: acc = c_0 / 2 T_0 + c_1 T_1, system by system (contiguous ranges)
    for (int sy = 0; sy < nsys; ++sy) {
        const int64_t off = PK->rp[row0[sy]] * b * b;
        const int64_t len = (PK->rp[row0[sy + 1]] - PK->rp[row0[sy]]) * b * b;
        for (int q = 0; q < rq.nq; ++q) {
            const double *c = rq.coef_tab + (size_t)q * n_pl * nsys;
            HIPCHECK(launch_axpby_to_f64(dtype, len, 0.5 * c[sy], (const char *)U0.p + off * esz,
                                         n_pl > 1 ? c[nsys + sy] : 0.0, (const char *)U1.p + off * esz,
                                         rq.acc[q] + off, st));
        }
    }
    const std::vector<int32_t> &tr0 = lp->usable ? lp->tile_row0 : plan->tile_row0;
    const int ntiles = (int)tr0.size() - 1;
    std::vector<int32_t> seg(nsys + 1);
    {
        int t = 0;
        for (int sy = 0; sy <= nsys; ++sy) {
            while (t < ntiles && tr0[t] < row0[sy]) ++t;
            seg[sy] = t;
        }
    }
    DevBuf dseg;
    upload(dseg, seg, st);
    // the last step k (product T_{k+1}) each system needs: n_pl(s) - 2
    DevBuf dlast;
    if (rq.sys_npl) {
        std::vector<int32_t> last(nsys);
        for (int sy = 0; sy < nsys; ++sy) last[sy] = (*rq.sys_npl)[sy] - 2;
        upload(dlast, last, st);
    }
    DevBuf part(sizeof(double) * (size_t)std::max(n_pl, 2) * std::max(ntiles, 256));
    DevBuf mom(sizeof(double) * (size_t)std::max(n_pl, 2) * nsys);
    double *pd = part.as<double>();
    const int tparts = 256;
    for (int sy = 0; sy < nsys; ++sy) {
        const int nbs = row0[sy + 1] - row0[sy];
        const int64_t *dg = PK->d_diag.as<int64_t>() + row0[sy];
        HIPCHECK(launch_trace(dtype, b, nbs, dg, U0.p, pd, tparts, st));
        HIPCHECK(launch_reduce_rows(1, tparts, pd, mom.as<double>() + sy, st));
        HIPCHECK(launch_trace(dtype, b, nbs, dg, U1.p, pd, tparts, st));
        HIPCHECK(launch_reduce_rows(1, tparts, pd, mom.as<double>() + nsys + sy, st));
    }
    void *ucur = U1.p, *uprev = U0.p;
    auto step = [&](int k) {
        Epilogue ep;
        ep.alpha = 2.0;
        ep.beta = -1.0;
        ep.prev = uprev;
        ep.nacc = rq.nq;
        ep.row_sys = rq.d_row_sys;
        ep.sys_last = rq.sys_npl ? dlast.as<int32_t>() : nullptr;
        ep.step = k;
        for (int q = 0; q < rq.nq; ++q) {
            ep.acc[q] = rq.acc[q];
            ep.coef_sys[q] = dcoef.as<double>() + ((size_t)q * n_pl + k + 1) * nsys;
        }
        ep.trace_partial = pd + (size_t)(k + 1) * ntiles;
        if (lp->usable)
            product_listed(ctx, dtype, lp, ucur, Bt.p, uprev, ep, rq.opmode, Bhi.p, Blo.p);
        else
            product(ctx, dtype, plan, ucur, Bt.p, uprev, ep);
        std::swap(ucur, uprev);
    };
    Timer tm(st);
    tm.start();
    if (n_pl > 2) step(1);  // eager: also settles per-kernel attributes before recording
    if (n_pl > 3) {
        if (rq.use_graph) {
            if (!ctx->capture_stream) HIPCHECK(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            ctx->stream = ctx->capture_stream;  // the products are recorded, not run
            try {
                HIPCHECK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed));
                for (int k = 2; k + 1 < n_pl; ++k) step(k);
                HIPCHECK(hipStreamEndCapture(ctx->stream, &graph));
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(ctx->stream, &g);
                if (g) (void)hipGraphDestroy(g);
                ctx->stream = st;
                throw;
            }
            ctx->stream = st;
            size_t nn = 0;
            (void)hipGraphGetNodes(graph, nullptr, &nn);
            rq.graph_nodes = (int)nn;
            hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (e == hipSuccess) e = hipGraphLaunch(exec, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (exec) (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
            HIPCHECK(e);
        } else {
            for (int k = 2; k + 1 < n_pl; ++k) step(k);
        }
    }
    rq.kernel_ms = tm.stop();
    if (n_pl > 2)
        HIPCHECK(launch_segment_sum(n_pl - 2, ntiles, nsys, dseg.as<int32_t>(), pd + 2 * (size_t)ntiles,
                                    mom.as<double>() + 2 * (size_t)nsys, st));
    if (rq.moments) {
        rq.moments->assign((size_t)n_pl * nsys, 0.0);
        HIPCHECK(hipMemcpyAsync(rq.moments->data(), mom.p, sizeof(double) * (size_t)n_pl * nsys, hipMemcpyDeviceToHost, st));
    }
    HIPCHECK(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------------------
// option handling
// ---------------------------------------------------------------------------

static chess_opts resolve_opts(const chess_opts *o) {
    chess_opts r;
    chess_default_opts(&r);
    if (o) r = *o;
    if (r.precision != CHESS_F64 && r.precision != CHESS_F32 && r.precision != CHESS_BF16 &&
        r.precision != CHESS_BF16X3)
        CHESS_THROW(CHESS_E_UNSUPPORTED, "precision %d", r.precision);
    if (r.smearing != CHESS_ERFC && r.smearing != CHESS_FERMI_DIRAC) CHESS_THROW(CHESS_E_ARG, "smearing %d", r.smearing);
    if (r.bounds_mode != CHESS_BOUNDS_GERSHGORIN && r.bounds_mode != CHESS_BOUNDS_LANCZOS &&
        r.bounds_mode != CHESS_BOUNDS_LEARNED && r.bounds_mode != CHESS_BOUNDS_LEARNED_LANCZOS)
        CHESS_THROW(CHESS_E_ARG, "bounds_mode %d", r.bounds_mode);
    const double deftol = r.precision == CHESS_F64 ? 1e-10 : r.precision == CHESS_BF16 ? 1e-4 : 1e-6;
    if (!(r.tol_fit > 0)) r.tol_fit = deftol;
    if (!(r.tol_fit_s > 0)) r.tol_fit_s = deftol;
    if (r.max_reexpand < 0) r.max_reexpand = 0;
    if (r.lanczos_steps <= 0) r.lanczos_steps = 40;
    if (!(r.eig_width > 0)) r.eig_width = 1e-3;
    if (!(r.bound_margin >= 0)) r.bound_margin = 0.02;
    if (!(r.kt_ratio > 1)) r.kt_ratio = 1.25;
    if (r.max_kt_halvings < 0) r.max_kt_halvings = 0;
    return r;
}

static void check_matrix(const chess_matrix *M, const char *what) {
    if (!M) CHESS_THROW(CHESS_E_ARG, "%s: null matrix", what);
    if (M->dtype != CHESS_F64) CHESS_THROW(CHESS_E_UNSUPPORTED, "%s: dtype must be CHESS_F64", what);
    if (!M->val) CHESS_THROW(CHESS_E_ARG, "%s: null values", what);
}

// Bounds of S for x^a with a possibly non-integer / negative: Gershgorin
// upper bound; Gershgorin lower bound when positive, else Lanczos.
static void s_bounds(chess_ctx *ctx, const Pattern *PS, const double *S, const chess_opts &o,
                     bool need_positive, double *lo, double *hi) {
    if (std::isfinite(o.s_bounds[0]) && std::isfinite(o.s_bounds[1])) {
        *lo = o.s_bounds[0];
        *hi = o.s_bounds[1];
    } else {
        double glo, ghi;
        gershgorin(ctx, PS, S, &glo, &ghi);
        *hi = ghi;
        *lo = glo;
        if (need_positive && glo <= 0) {
            double tmin, tmax, rmin, rmax;
            lanczos(ctx, PS, S, o.lanczos_steps, &tmin, &tmax, &rmin, &rmax);
            *lo = tmin - rmin - o.bound_margin * (tmax - tmin);
        }
    }
    if (!(*hi > *lo)) CHESS_THROW(CHESS_E_ARG, "empty spectral interval [%g, %g]", *lo, *hi);
    if (need_positive && !(*lo > 0)) CHESS_THROW(CHESS_E_NOT_SPD, "lower spectral bound %g is not positive", *lo);
}

// |t_k| <= n (1 + 1e-2) holds whenever the spectrum is inside the bounds.
static bool growth_ok(const std::vector<double> &t, int64_t n) {
    for (double v : t)
        if (!std::isfinite(v) || std::fabs(v) > 1.01 * (double)n) return false;
    return true;
}

// x^a by the chain on S~ (U-form accumulator -> acc, transposed storage).
// The bounds are judged by the growth test and Eq. 6 on at least
// penalty_degree(n) moments: a shorter series is first checked on a
// moments-only chain of that length, a longer one on its own moments.  A
// failed growth test widens both sides by 10 % of the width (its side is not
// trusted when both bounds may be off, as for a default guess); a failed
// Eq. 6 (an eigenvalue at or within about 1 % of a bound) moves only the
// penalty's side, by 2.5 % of the width, since x^a is steepest at the lower
// bound, where a larger step costs terms and precision.  The lower bound at
// most halves, so it stays positive.  The check chain multiplies operands in the storage
// precision (float32 in the bfloat16 forms).
struct PowerResult {
    double lo, hi;
    int n_pl;
    int reexp;
    double kernel_ms;
    int variant = -1;
    double penalty = NAN;  // Tr W^p for the final bounds (NaN if not evaluated)
    int check_terms = 0;   // moments the final bounds were judged on
    int products = 0;      // product launches, check chains included
};

// The widening of a matrix power's bounds after a failed check (see above).
static void widen_power(const hostmath::BoundsCheck &chk, double *lo, double *hi) {
    const double w = *hi - *lo;
    const int side = chk.valid ? chk.side : 0;
    const double step = chk.valid ? 0.025 : 0.1;
    if (side <= 0) *lo = std::max(*lo - step * w, 0.5 * *lo);
    if (side >= 0) *hi += step * w;
}

static PowerResult power_chain(chess_ctx *ctx, const Pattern *PS, const double *S,
                               const Pattern *PK, const std::vector<double> &powers,
                               const chess_opts &o, int n_pl_fixed, double tol, double *const *acc,
                               double lo, double hi) {
    hipStream_t st = ctx->stream;
    DevBuf St(sizeof(double) * (size_t)PS->nnzb * PS->b * PS->b);
    PowerResult r{lo, hi, 0, 0, 0.0};
    const int64_t n = PK->n();
    const int n_check = hostmath::penalty_degree(n);
    for (int attempt = 0;; ++attempt) {
        double sigma, tau;
        hostmath::scale_shift(r.lo, r.hi, &sigma, &tau);
        HIPCHECK(launch_scale_shift(PS->b, PS->nnzb, PS->d_brow.as<int32_t>(), PS->d_ci.as<int32_t>(), S, St.as<double>(), sigma, tau, st));
        int n_pl = n_pl_fixed;
        if (n_pl <= 0) {
            n_pl = 1;
            for (double a : powers) {
                const int m = hostmath::degree([a](double x) { return std::pow(x, a); }, r.lo, r.hi, tol, 8, 20000);
                if (m < 0) CHESS_THROW(CHESS_E_NOCONV, "no degree up to 20000 reaches tol_fit %g for x^%g", tol, a);
                n_pl = std::max(n_pl, m);
            }
        }
        hostmath::BoundsCheck chk;
        if (n_pl < n_check) {
            // too few terms for Eq. 6: judge the bounds on a moments-only
            // chain of n_check terms before summing the series
            std::vector<double> cm;
            ChainRequest cq;
            cq.label = "S check chain";
            cq.PM = PS;
            cq.Mt = St.as<double>();
            cq.PK = PK;
            cq.n_pl = n_check;
            cq.dtype = storage_dtype(o.precision);
            // the storage precision's own operands, also in the bfloat16
            // forms: rounding the operands to bfloat16 puts noise of order
            // 0.01 sqrt(n) on Tr W^p, past the threshold of 0.5 at several
            // thousand rows
            cq.opmode = 0;
            cq.moments = &cm;
            run_chain(ctx, cq);
            r.kernel_ms += cq.kernel_ms;
            r.products += cq.products;
            chk = hostmath::bounds_check(cm, n);
        }
        if (n_pl >= n_check || chk.ok) {
            std::vector<double> coef((size_t)powers.size() * n_pl);
            for (size_t q = 0; q < powers.size(); ++q) {
                const double a = powers[q];
                auto c = hostmath::cheb_coeffs([a](double x) { return std::pow(x, a); }, r.lo, r.hi, n_pl);
                std::copy(c.begin(), c.end(), coef.begin() + q * n_pl);
            }
            std::vector<double> mom;
            ChainRequest rq;
            rq.label = "S chain";
            rq.PM = PS;
            rq.Mt = St.as<double>();
            rq.PK = PK;
            rq.n_pl = n_pl;
            rq.nq = (int)powers.size();
            rq.coef = coef.data();
            for (size_t q = 0; q < powers.size(); ++q) rq.acc[q] = acc[q];
            rq.dtype = storage_dtype(o.precision);
            rq.opmode = operand_mode(o.precision);
            rq.moments = &mom;
            run_chain(ctx, rq);
            r.kernel_ms += rq.kernel_ms;
            r.products += rq.products;
            r.variant = rq.variant;
            if (n_pl >= n_check) chk = hostmath::bounds_check(mom, n);
        }
        r.n_pl = n_pl;
        r.penalty = chk.penalty;
        r.check_terms = std::max(n_pl, n_check);
        if (chk.ok) break;
        if (attempt >= o.max_reexpand)
            CHESS_THROW(CHESS_E_BOUNDS, "spectral bounds [%g, %g] still fail after %d widenings", r.lo, r.hi, attempt);
        widen_power(chk, &r.lo, &r.hi);
        r.reexp++;
    }
    return r;
}

static void transpose_into(chess_ctx *ctx, const Pattern *P, const double *in, double *out) {
    HIPCHECK(launch_scatter_blocks(0, P->b, P->nnzb, P->d_tmap.as<int64_t>(), in, out, 1, ctx->stream));
}

static void require_same(const Pattern *a, const Pattern *b, const char *what) {
    if (a != b) CHESS_THROW(CHESS_E_PATTERN, "%s: output must be allocated on exactly the given pattern", what);
}

static void set_err(chess_ctx *ctx, const Error &e) { ctx->err = e.msg; }

// Orthogonal frame: X^T (accX, transposed storage), X, and H' on PH.
struct Frame {
    DevBuf accX, X, Hp;
    PowerResult s;
    // the interval of S the call started from (given, or Gershgorin/Lanczos),
    // before any widening by the checks: the predictor's features describe
    // the spectrum of S with it, as in its training data
    double s_lo0 = NAN, s_hi0 = NAN;
    double ms_s = 0, ms_transform = 0;
};

static void build_frame(chess_ctx *ctx, const Pattern *PH, const double *H, const Pattern *PS,
                        const double *S, const Pattern *PK, const chess_opts &o, Frame &F) {
    hipStream_t st = ctx->stream;
    Timer t(st);
    t.start();
    const size_t xbytes = sizeof(double) * (size_t)PK->nnzb * PK->b * PK->b;
    F.accX.alloc(xbytes);
    if (o.sinvhalf_in) {
        // S^-1/2 from an earlier call (Sec. "Performance": in an SCF cycle S
        // does not change): no S chain; its bounds are those given, if any
        transpose_into(ctx, PK, (const double *)o.sinvhalf_in, F.accX.as<double>());
        F.s = PowerResult{o.s_bounds[0], o.s_bounds[1], 0, 0, 0.0, -1};
        F.s_lo0 = o.s_bounds[0];
        F.s_hi0 = o.s_bounds[1];
    } else {
        double slo, shi;
        s_bounds(ctx, PS, S, o, true, &slo, &shi);
        F.s_lo0 = slo;
        F.s_hi0 = shi;
        double *accs[1] = {F.accX.as<double>()};
        F.s = power_chain(ctx, PS, S, PK, {-0.5}, o, o.n_pl_s, o.tol_fit_s, accs, slo, shi);
    }
    F.ms_s = t.stop();
    t.start();
    const EmbedMap *eh = get_embed(ctx, PH, PK, "H in the kernel pattern");
    (void)eh;
    // Z^T = P_K o (X^T H^T): A = X^T (= accX), Bt = H
    DevBuf ZT(sizeof(double) * (size_t)PK->nnzb * PK->b * PK->b);
    product(ctx, 0, get_plan(ctx, PK, PH, PK, 0), F.accX.p, H, ZT.p, Epilogue{});
    // X = (accX)^T
    F.X.alloc(ZT.bytes);
    transpose_into(ctx, PK, F.accX.as<double>(), F.X.as<double>());
    // H' = P_H o (X Z): A = X, Bt = Z^T; then symmetrise
    DevBuf Hraw(sizeof(double) * (size_t)PH->nnzb * PH->b * PH->b);
    product(ctx, 0, get_plan(ctx, PK, PK, PH, 0), F.X.p, ZT.p, Hraw.p, Epilogue{});
    F.Hp.alloc(Hraw.bytes);
    HIPCHECK(launch_symmetrize(PH->b, PH->nnzb, PH->d_tmap.as<int64_t>(), Hraw.as<double>(), F.Hp.as<double>(), st));
    if (o.sinvhalf_out) HIPCHECK(hipMemcpyAsync(o.sinvhalf_out, F.X.p, xbytes, hipMemcpyDeviceToDevice, st));
    F.ms_transform = t.stop();
}

static void h_bounds(chess_ctx *ctx, const Pattern *PH, const double *Hp, const chess_opts &o,
                     double *lo, double *hi) {
    if (std::isfinite(o.bounds[0]) && std::isfinite(o.bounds[1])) {
        *lo = o.bounds[0];
        *hi = o.bounds[1];
    } else if (o.bounds_mode == CHESS_BOUNDS_LANCZOS) {
        double tmin, tmax, rmin, rmax;
        lanczos(ctx, PH, Hp, o.lanczos_steps, &tmin, &tmax, &rmin, &rmax);
        const double w = tmax - tmin;
        *lo = tmin - rmin - o.bound_margin * w;
        *hi = tmax + rmax + o.bound_margin * w;
    } else {
        gershgorin(ctx, PH, Hp, lo, hi);
    }
    if (!(*hi > *lo)) CHESS_THROW(CHESS_E_ARG, "empty spectral interval [%g, %g]", *lo, *hi);
}

// ---------------------------------------------------------------------------
// learned predictor: features of H', network inference
// ---------------------------------------------------------------------------

// The 64 features (all from H' on its pattern, cheap next to the chain):
//   0 c, 1 w (centre and half width of the Gershgorin interval of H'),
//   2-3 bounds of S, 4 kT, 5 kT / w, 6 N_e / n, 7 log n, 8 b / 9,
//   9-16 t_k / n, k = 1..8, moments Tr T_k((H' - c) / w) from 7 chain steps,
//   17-40 histogram of the diagonal (d - c) / w over [-1, 1] (fractions),
//   41-56 histogram of the Gershgorin radii R / w over [0, 1] (fractions),
//   57-58 mean and standard deviation of (d - c) / w, 59-60 mean and max of
//   R / w, 61-62 min and max of (d - c) / w,
//   63 (mu_0 - c) / w with mu_0 solving N(mu) = N_e for the 9-term expansion
//      of a broad occupation (kT = w / 4) from the same moments.
struct Features {
    float f[kMlpIn];
    double g_lo = 0, g_hi = 0;
};

static void compute_features(chess_ctx *ctx, const Pattern *PH, const double *Hp, const Pattern *PK,
                             double s_lo, double s_hi, double n_e, double kT, Features &fe) {
    static_assert(kMlpIn == 64 && kDiagBins == 24 && kRadBins == 16, "feature layout");
    hipStream_t st = ctx->stream;
    const int b = PH->b;
    const int64_t n = PH->n();
    double g_lo, g_hi;
    gershgorin(ctx, PH, Hp, &g_lo, &g_hi);
    const double c = 0.5 * (g_lo + g_hi), w = 0.5 * (g_hi - g_lo);
    if (!(w > 0)) CHESS_THROW(CHESS_E_ARG, "features: Gershgorin interval of H' is empty");
    const int parts = row_feature_parts(b, PH->nb);
    DevBuf hist(sizeof(uint32_t) * (kDiagBins + kRadBins)), part(sizeof(double) * 6 * (size_t)parts);
    HIPCHECK(launch_zero(hist.p, hist.bytes, st));
    HIPCHECK(launch_row_features(b, PH->nb, PH->d_rp.as<int64_t>(), PH->d_ci.as<int32_t>(), Hp, c, w,
                                 hist.as<uint32_t>(), part.as<double>(), st));
    std::vector<uint32_t> hh(kDiagBins + kRadBins);
    std::vector<double> pp(6 * (size_t)parts);
    HIPCHECK(hipMemcpyAsync(hh.data(), hist.p, hist.bytes, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(pp.data(), part.p, pp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    // moments of (H' - c) / w
    DevBuf Ht(sizeof(double) * (size_t)PH->nnzb * b * b);
    HIPCHECK(launch_scale_shift(b, PH->nnzb, PH->d_brow.as<int32_t>(), PH->d_ci.as<int32_t>(), Hp,
                                Ht.as<double>(), 1.0 / w, c, st));
    std::vector<double> mom;
    ChainRequest rq;
    rq.label = "feature moments";
    rq.PM = PH;
    rq.Mt = Ht.as<double>();
    rq.PK = PK;
    rq.n_pl = 9;
    rq.dtype = 0;
    rq.moments = &mom;
    run_chain(ctx, rq);  // synchronises the stream
    double sd = 0, sd2 = 0, sr = 0, mr = -1e300, mnd = 1e300, mxd = -1e300;
    for (int q = 0; q < parts; ++q) {
        const double *o = &pp[6 * (size_t)q];
        sd += o[0];
        sd2 += o[1];
        sr += o[2];
        mr = std::max(mr, o[3]);
        mnd = std::min(mnd, o[4]);
        mxd = std::max(mxd, o[5]);
    }
    const double dn = (double)n;
    hostmath::CountFunction N;
    N.init(mom, g_lo, g_hi, 0.25 * w, 0);
    double mu0 = c;
    int it = 0;
    if (!hostmath::bisect_mu(N, n_e, 1e-9 * std::max(1.0, n_e), g_lo - 4 * w, g_hi + 4 * w, &mu0, &it)) mu0 = c;
    float *f = fe.f;
    f[0] = (float)c;
    f[1] = (float)w;
    f[2] = (float)s_lo;
    f[3] = (float)s_hi;
    f[4] = (float)kT;
    f[5] = (float)(kT / w);
    f[6] = (float)(n_e / dn);
    f[7] = (float)std::log(dn);
    f[8] = (float)(b / 9.0);
    for (int k = 1; k <= 8; ++k) f[8 + k] = (float)(mom[k] / dn);
    for (int q = 0; q < kDiagBins; ++q) f[17 + q] = (float)(hh[q] / dn);
    for (int q = 0; q < kRadBins; ++q) f[41 + q] = (float)(hh[kDiagBins + q] / dn);
    const double mean_d = sd / dn;
    f[57] = (float)mean_d;
    f[58] = (float)std::sqrt(std::max(0.0, sd2 / dn - mean_d * mean_d));
    f[59] = (float)(sr / dn);
    f[60] = (float)mr;
    f[61] = (float)mnd;
    f[62] = (float)mxd;
    f[63] = (float)((mu0 - c) / w);
    fe.g_lo = g_lo;
    fe.g_hi = g_hi;
}

// Network outputs for one feature vector, mapped back to energies:
// out = {eps_min, eps_max, mu} = c + w * y.
static void predict(chess_ctx *ctx, const Features &fe, double out[3]) {
    if (!ctx->model.loaded) CHESS_THROW(CHESS_E_ARG, "no model loaded (chess_model_load)");
    hipStream_t st = ctx->stream;
    DevBuf x(sizeof(float) * kMlpIn), y(sizeof(float) * kMlpOut);
    HIPCHECK(hipMemcpyAsync(x.p, fe.f, sizeof(float) * kMlpIn, hipMemcpyHostToDevice, st));
    HIPCHECK(launch_mlp_forward(ctx->model.params.as<float>(), ctx->model.norm.as<float>(), x.as<float>(),
                                1, nullptr, y.as<float>(), st));
    float yh[kMlpOut];
    HIPCHECK(hipMemcpyAsync(yh, y.p, sizeof(yh), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    const double c = 0.5 * (fe.g_lo + fe.g_hi), w = 0.5 * (fe.g_hi - fe.g_lo);
    for (int q = 0; q < kMlpOut; ++q) out[q] = c + w * (double)yh[q];
}

static hostmath::Fn occupation(int smearing, double mu, double kT) {
    if (smearing == CHESS_ERFC) return [mu, kT](double e) { return hostmath::occ_erfc(e, mu, kT); };
    return [mu, kT](double e) { return hostmath::occ_fd(e, mu, kT); };
}

// K = P_K o (X P_K o (K' X)) from accK = K'^T; Tr(KS).
static double post_transform(chess_ctx *ctx, const Pattern *PK, const Frame &F, const double *accK,
                             const Pattern *PS, const double *S, double *Kout) {
    const size_t bytes = sizeof(double) * (size_t)PK->nnzb * PK->b * PK->b;
    DevBuf Kp(bytes), WT(bytes);
    transpose_into(ctx, PK, accK, Kp.as<double>());
    // W^T = P_K o (X^T K'^T): A = X^T (accX), Bt = K'
    product(ctx, 0, get_plan(ctx, PK, PK, PK, 0), F.accX.p, Kp.p, WT.p, Epilogue{});
    // K = P_K o (X W): A = X, Bt = W^T
    product(ctx, 0, get_plan(ctx, PK, PK, PK, 0), F.X.p, WT.p, Kout, Epilogue{});
    // Tr(K S) = sum over S blocks (J, I) of <K(I, J), S(J, I)^T>
    const EmbedMap *es = get_embed(ctx, PS, PK, "S in the kernel pattern");
    const int nparts = 256;
    DevBuf part(sizeof(double) * (nparts + 1));
    HIPCHECK(launch_trace_product(PK->b, PS->nnzb, es->d_map_t.as<int64_t>(), Kout, S, part.as<double>(), nparts, ctx->stream));
    HIPCHECK(launch_reduce_rows(1, nparts, part.as<double>(), part.as<double>() + nparts, ctx->stream));
    double tr;
    HIPCHECK(hipMemcpyAsync(&tr, part.as<double>() + nparts, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(hipStreamSynchronize(ctx->stream));
    return tr;
}

// HOMO / LUMO estimates from the moments of a density-kernel chain (Sec.
// "Extraction of selected eigenvalues"): eigenvalue N solves N(e) = N - 1/2,
// so with N_h = ceil(N_e) occupied states the HOMO solves N(e) = N_h - 1/2
// and the LUMO N(e) = N_h + 1/2.  NaN past either end of the n states.
static void homo_lumo(const hostmath::CountFunction &N, double n_e, double n_states, double lo,
                      double hi, double kT, double *homo, double *lumo) {
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const double nh = std::ceil(n_e - 1e-9);
    const double tol = 1e-10 * std::max(1.0, n_e);
    int it = 0;
    *homo = *lumo = nan;
    if (nh >= 1 && !hostmath::bisect_mu(N, nh - 0.5, tol, lo - 20 * kT, hi + 20 * kT, homo, &it))
        *homo = nan;
    if (nh + 1 <= n_states && !hostmath::bisect_mu(N, nh + 0.5, tol, lo - 20 * kT, hi + 20 * kT, lumo, &it))
        *lumo = nan;
}

static void fill_info_defaults(chess_info *info) {
    if (!info) return;
    std::memset(info, 0, sizeof(*info));
    const double nan = std::numeric_limits<double>::quiet_NaN();
    info->mu = info->lo = info->hi = info->s_lo = info->s_hi = nan;
    info->tr_ks = info->ne_chain = info->penalty = info->s_penalty = nan;
    info->pred_lo = info->pred_hi = info->pred_mu = nan;
    info->energy = info->energy_wide = info->homo = info->lumo = nan;
    info->kernel_variant = -1;
}

// E = Tr(p(H') H') from the moments t_k = Tr T_k(H~), one more than the
// coefficients c (Sec. "Fermi Operator Expansion" compares E for two widths).
// H' = H~ / sigma + tau I, and the recursion 2 x T_k = T_{k+1} + T_{k-1} gives
// Tr(T_0 H~) = t_1, Tr(T_k H~) = (t_{k+1} + t_{k-1}) / 2; the truncated chain
// keeps every diagonal block, so this holds for it exactly.
static double energy_from_moments(const std::vector<double> &c, const std::vector<double> &t, double lo,
                                  double hi) {
    double sigma, tau;
    hostmath::scale_shift(lo, hi, &sigma, &tau);
    const int n = (int)c.size();
    if ((int)t.size() < n + 1) CHESS_THROW(CHESS_E_ARG, "energy needs %d moments", n + 1);
    auto tr = [&](int k) {
        const double g = k == 0 ? t[1] : 0.5 * (t[k + 1] + t[k - 1]);
        return g / sigma + tau * t[k];
    };
    double e = 0.5 * c[0] * tr(0);
    for (int k = 1; k < n; ++k) e += c[k] * tr(k);
    return e;
}

static void fermi_operator(chess_ctx *ctx, const chess_matrix *H, const chess_matrix *S,
                           const chess_pattern *pattern, double n_e, double kT,
                           chess_matrix *K_out, chess_info *info, const chess_opts *opts) {
    const double t_begin = now_ms();
    chess_opts o = resolve_opts(opts);
    check_matrix(H, "H");
    check_matrix(S, "S");
    check_matrix(K_out, "K_out");
    if (!(kT > 0)) CHESS_THROW(CHESS_E_ARG, "kT must be positive");
    const Pattern *PH = get_pattern(ctx, &H->pat, "H pattern");
    const Pattern *PS = get_pattern(ctx, &S->pat, "S pattern");
    const Pattern *PK = get_pattern(ctx, pattern, "kernel pattern");
    require_same(get_pattern(ctx, &K_out->pat, "K_out pattern"), PK, "K_out");
    if (PH->nb != PK->nb || PS->nb != PK->nb || PH->b != PK->b || PS->b != PK->b)
        CHESS_THROW(CHESS_E_ARG, "H, S and the pattern differ in size or block edge");
    const int64_t n = PK->n();
    if (!(n_e >= 0 && n_e <= (double)n)) CHESS_THROW(CHESS_E_ARG, "n_electrons %g outside [0, %lld]", n_e, (long long)n);
    get_embed(ctx, PH, PK, "H in the kernel pattern");
    get_embed(ctx, PS, PK, "S in the kernel pattern");
    hipStream_t st = ctx->stream;
    const double t_setup = now_ms();

    Frame F;
    build_frame(ctx, PH, H->val ? (const double *)H->val : nullptr, PS, (const double *)S->val, PK, o, F);
    const int b = PK->b;
    const int dtype = storage_dtype(o.precision);
    const int64_t nK = PK->nnzb * b * b;
    double lo, hi;
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const bool given = std::isfinite(o.bounds[0]) && std::isfinite(o.bounds[1]);
    bool learned = false;
    int fallback = 0;
    double pred[3] = {nan, nan, nan};
    double br[2] = {o.mu_bracket[0], o.mu_bracket[1]};
    const bool br_given = std::isfinite(br[0]) && std::isfinite(br[1]);
    Features fe;
    double ms_learned = 0.0;
    // interval taken when the predicted one is rejected
    double fb_lo = nan, fb_hi = nan;
    const bool with_model = o.bounds_mode == CHESS_BOUNDS_LEARNED || o.bounds_mode == CHESS_BOUNDS_LEARNED_LANCZOS;
    if (!given && with_model) {
        // predicted bounds widened by the model's margins (never beyond the
        // Gershgorin interval) and a predicted mu bracket; Eq. 6 and the
        // growth test still judge the bounds, bisection still judges mu
        const double t0 = now_ms();
        if (!(std::isfinite(F.s_lo0) && std::isfinite(F.s_hi0)))
            CHESS_THROW(CHESS_E_ARG, "learned bounds with a given S^-1/2 need s_bounds");
        compute_features(ctx, PH, F.Hp.as<double>(), PK, F.s_lo0, F.s_hi0, n_e, kT, fe);
        predict(ctx, fe, pred);
        const Model &M = ctx->model;
        const double w = 0.5 * (fe.g_hi - fe.g_lo);
        lo = std::max(fe.g_lo, pred[0] - M.margin_lo * w);
        hi = std::min(fe.g_hi, pred[1] + M.margin_hi * w);
        fb_lo = fe.g_lo;
        fb_hi = fe.g_hi;
        if (o.bounds_mode == CHESS_BOUNDS_LEARNED_LANCZOS) {
            // each side from whichever estimate is tighter there; the
            // Lanczos interval alone is the fallback
            chess_opts ol = o;
            ol.bounds_mode = CHESS_BOUNDS_LANCZOS;
            h_bounds(ctx, PH, F.Hp.as<double>(), ol, &fb_lo, &fb_hi);
            lo = std::max(lo, fb_lo);
            hi = std::min(hi, fb_hi);
        }
        if (hi > lo) {
            learned = true;
        } else {
            lo = fb_lo;
            hi = fb_hi;
            fallback |= 1;
        }
        if (!br_given) {
            br[0] = pred[2] - M.mu_half * w;
            br[1] = pred[2] + M.mu_half * w;
        }
        ms_learned = now_ms() - t0;
    } else {
        h_bounds(ctx, PH, F.Hp.as<double>(), o, &lo, &hi);
    }

    DevBuf Ht(sizeof(double) * (size_t)PH->nnzb * b * b);
    DevBuf accK(sizeof(double) * (size_t)nK);
    DevBuf hist;
    std::vector<double> mom;
    int n_pl = 0, reexp = 0, passes = 0;
    double penalty = std::numeric_limits<double>::quiet_NaN();
    double ms_chain = 0.0, kernel_ms = 0.0, kernel_ms_acc = 0.0;
    int variant = -1, variant_moments = -1, tile_rows = 0, moment_products = 0, products = 0;
    bool have_hist = false;
    Timer tm(st);
    // Width check of Sec. "Fermi Operator Expansion" (adapt_kt): the chain
    // runs one term longer so that E = Tr(K' H') follows from its moments;
    // E at kT and E' at kt_ratio kT (each with its own mu) are compared and
    // kT is halved (a new expansion) while they differ by more than tol_energy.
    const int extra = o.adapt_kt ? 1 : 0;
    double energy = nan, energy_wide = nan, ms_mu = 0.0, mu = o.mu;
    int halvings = 0, iters = 0;
    for (;;) {
    for (int attempt = 0;; ++attempt) {
        double sigma, tau;
        hostmath::scale_shift(lo, hi, &sigma, &tau);
        n_pl = o.n_pl;
        if (n_pl <= 0) {
            n_pl = hostmath::degree(occupation(o.smearing, tau, kT), lo, hi, o.tol_fit, 8, 20000);
            if (n_pl < 0) CHESS_THROW(CHESS_E_NOCONV, "no degree up to 20000 reaches tol_fit %g", o.tol_fit);
        }
        HIPCHECK(launch_scale_shift(b, PH->nnzb, PH->d_brow.as<int32_t>(), PH->d_ci.as<int32_t>(), F.Hp.as<double>(), Ht.as<double>(), sigma, tau, st));
        have_hist = false;
        if (o.store_history && !std::isfinite(o.mu)) {
            size_t freeb = 0, totalb = 0;
            HIPCHECK(hipMemGetInfo(&freeb, &totalb));
            const size_t need = vbytes(PK, dtype) * (size_t)(n_pl + extra);
            if (need + ((size_t)1 << 30) < freeb) {
                try {
                    hist.alloc(need);
                    have_hist = true;
                } catch (const Error &) {
                    have_hist = false;
                }
            }
        }
        tm.start();
        ChainRequest rq;
        rq.label = "H chain";
        rq.PM = PH;
        rq.Mt = Ht.as<double>();
        rq.PK = PK;
        rq.n_pl = n_pl + extra;
        rq.dtype = dtype;
        rq.opmode = operand_mode(o.precision);
        rq.moments = &mom;
        std::vector<double> c_fixed;
        if (std::isfinite(o.mu)) {
            // mu given: one accumulating pass (the extra term has weight 0)
            c_fixed = hostmath::cheb_coeffs(occupation(o.smearing, o.mu, kT), lo, hi, n_pl);
            c_fixed.resize(n_pl + extra, 0.0);
            rq.nq = 1;
            rq.coef = c_fixed.data();
            rq.acc[0] = accK.as<double>();
        }
        rq.hist = have_hist ? hist.p : nullptr;
        run_chain(ctx, rq);
        ms_chain += tm.stop();
        kernel_ms += rq.kernel_ms;
        if (rq.nq > 0) kernel_ms_acc += rq.kernel_ms;
        else variant_moments = rq.variant;
        if (rq.nq == 0) moment_products += rq.products;
        products += rq.products;
        variant = rq.variant;
        tile_rows = rq.tile_rows;
        passes++;
        const hostmath::BoundsCheck chk = hostmath::bounds_check(mom, n);
        penalty = chk.penalty;
        if (chk.ok) break;
        if (learned) {
            // predicted bounds rejected: fall back to the Gershgorin (or,
            // combined with Lanczos, the Lanczos) interval
            lo = fb_lo;
            hi = fb_hi;
            learned = false;
            fallback |= 1;
            reexp++;
            continue;
        }
        if (attempt >= o.max_reexpand) CHESS_THROW(CHESS_E_BOUNDS, "spectral bounds [%g, %g] still fail after %d widenings", lo, hi, attempt);
        // Eq. 6 sign tells which side: positive -> an eigenvalue below lo
        hostmath::widen(chk.side, &lo, &hi);
        reexp++;
    }
    // mu search on the moments
    const std::vector<double> mom_e(mom);  // with the extra moment
    mom.resize(n_pl);
    const double t_mu0 = now_ms();
    mu = o.mu;
    iters = 0;
    hostmath::CountFunction N;
    N.init(mom, lo, hi, kT, o.smearing == CHESS_ERFC ? 0 : 1);
    if (!std::isfinite(mu)) {
        const double tol_ne = o.tol_ne > 0 ? o.tol_ne : 1e-8 * n_e;
        bool found = false;
        if (std::isfinite(br[0]) && std::isfinite(br[1])) {
            found = hostmath::bisect_mu(N, n_e, tol_ne, br[0], br[1], &mu, &iters);
            if (!found && !br_given) fallback |= 2;
        }
        if (!found) {
            int it2 = 0;
            found = hostmath::bisect_mu(N, n_e, tol_ne, lo - 20 * kT, hi + 20 * kT, &mu, &it2);
            iters += it2;
        }
        if (!found) CHESS_THROW(CHESS_E_NOCONV, "N(mu) does not bracket %g electrons", n_e);
    }
    ms_mu += now_ms() - t_mu0;
    if (!o.adapt_kt) break;
    {
        const std::vector<double> c1 = hostmath::cheb_coeffs(occupation(o.smearing, mu, kT), lo, hi, n_pl);
        energy = energy_from_moments(c1, mom_e, lo, hi);
        const double kt2 = o.kt_ratio * kT;
        hostmath::CountFunction N2;
        N2.init(mom, lo, hi, kt2, o.smearing == CHESS_ERFC ? 0 : 1);
        double mu2 = 0.0;
        int it2 = 0;
        const double tol_ne = o.tol_ne > 0 ? o.tol_ne : 1e-8 * n_e;
        if (!hostmath::bisect_mu(N2, n_e, tol_ne, lo - 20 * kt2, hi + 20 * kt2, &mu2, &it2))
            CHESS_THROW(CHESS_E_NOCONV, "N(mu) at the second width does not bracket %g electrons", n_e);
        const std::vector<double> c2 = hostmath::cheb_coeffs(occupation(o.smearing, mu2, kt2), lo, hi, n_pl);
        energy_wide = energy_from_moments(c2, mom_e, lo, hi);
        const double tol_e = o.tol_energy > 0 ? o.tol_energy : 1e-4 * n_e;
        if (std::fabs(energy - energy_wide) <= tol_e || halvings >= o.max_kt_halvings) break;
        kT *= 0.5;
        halvings++;
        // a bracket predicted for the first width does not hold for the next
        if (!br_given) br[0] = br[1] = nan;
    }
    }
    double homo = nan, lumo = nan;
    {
        hostmath::CountFunction Ng;
        Ng.init(mom, lo, hi, kT, o.smearing == CHESS_ERFC ? 0 : 1);
        homo_lumo(Ng, n_e, (double)n, lo, hi, kT, &homo, &lumo);
    }
    const std::vector<double> c = hostmath::cheb_coeffs(occupation(o.smearing, mu, kT), lo, hi, n_pl);
    double ne_chain = 0.5 * c[0] * mom[0];
    for (int j = 1; j < n_pl; ++j) ne_chain += c[j] * mom[j];
    if (!std::isfinite(o.mu)) {
        tm.start();
        if (have_hist) {
            DevBuf dc(sizeof(double) * n_pl);
            std::vector<double> cc(c);
            cc[0] *= 0.5;  // T_0 enters with c_0/2
            HIPCHECK(hipMemcpyAsync(dc.p, cc.data(), sizeof(double) * n_pl, hipMemcpyHostToDevice, st));
            HIPCHECK(launch_recombine(dtype, nK, n_pl, hist.p, dc.as<double>(), accK.as<double>(), st));
            HIPCHECK(hipStreamSynchronize(st));
        } else {
            ChainRequest rq;
            rq.label = "H chain (accumulate)";
            rq.PM = PH;
            rq.Mt = Ht.as<double>();
            rq.PK = PK;
            rq.n_pl = n_pl;
            rq.dtype = dtype;
            rq.opmode = operand_mode(o.precision);
            rq.nq = 1;
            rq.coef = c.data();
            rq.acc[0] = accK.as<double>();
            run_chain(ctx, rq);
            kernel_ms += rq.kernel_ms;
            kernel_ms_acc += rq.kernel_ms;
            products += rq.products;
            variant = rq.variant;
            passes++;
        }
        ms_chain += tm.stop();
    }
    hist.release();
    Ht.release();
    const double t_post0 = now_ms();
    const double trks = post_transform(ctx, PK, F, accK.as<double>(), PS, (const double *)S->val, (double *)K_out->val);
    const double t_end = now_ms();
    if (info) {
        info->mu = mu;
        info->lo = lo;
        info->hi = hi;
        info->s_lo = F.s.lo;
        info->s_hi = F.s.hi;
        info->tr_ks = trks;
        info->ne_chain = ne_chain;
        info->penalty = penalty;
        info->n_pl = n_pl;
        info->n_pl_s = F.s.n_pl;
        info->passes = passes;
        info->bisect_iters = iters;
        info->reexpansions = reexp + F.s.reexp;
        info->s_penalty = F.s.penalty;
        info->s_check_terms = F.s.check_terms;
        info->chain_steps = products + F.s.products;
        info->moment_products = moment_products;
        info->ms_total = t_end - t_begin;
        info->ms_setup = t_setup - t_begin;
        info->ms_s_chain = F.ms_s;
        info->ms_transform = F.ms_transform;
        info->ms_h_chain = ms_chain;
        info->ms_mu = ms_mu;
        info->ms_post = t_end - t_post0;
        info->ms_chain_kernel = kernel_ms;
        info->ms_chain_kernel_acc = kernel_ms_acc;
        info->kernel_variant_moments = variant_moments;
        info->tile_rows = tile_rows;
        info->kernel_variant = variant;
        info->pred_lo = pred[0];
        info->pred_hi = pred[1];
        info->pred_mu = pred[2];
        info->fallback = fallback;
        info->ms_learned = ms_learned;
        info->energy = energy;
        info->energy_wide = energy_wide;
        info->kt_used = kT;
        info->kt_halvings = halvings;
        info->homo = homo;
        info->lumo = lumo;
    }
}

static void matrix_power(chess_ctx *ctx, const chess_matrix *S, double a,
                         const chess_pattern *pattern, chess_matrix *out, chess_info *info,
                         const chess_opts *opts) {
    const double t0 = now_ms();
    chess_opts o = resolve_opts(opts);
    check_matrix(S, "S");
    check_matrix(out, "Sa_out");
    if (!std::isfinite(a)) CHESS_THROW(CHESS_E_ARG, "power must be finite");
    const Pattern *PS = get_pattern(ctx, &S->pat, "S pattern");
    const Pattern *PK = get_pattern(ctx, pattern, "output pattern");
    require_same(get_pattern(ctx, &out->pat, "Sa_out pattern"), PK, "Sa_out");
    get_embed(ctx, PS, PK, "S in the output pattern");
    const bool need_pos = !(a == std::floor(a) && a >= 0);
    double lo, hi;
    s_bounds(ctx, PS, (const double *)S->val, o, need_pos, &lo, &hi);
    if (o.n_pl > 0) o.n_pl_s = o.n_pl;
    DevBuf acc(sizeof(double) * (size_t)PK->nnzb * PK->b * PK->b);
    double *accs[1] = {acc.as<double>()};
    PowerResult r = power_chain(ctx, PS, (const double *)S->val, PK, {a}, o, o.n_pl_s, o.tol_fit_s, accs, lo, hi);
    transpose_into(ctx, PK, acc.as<double>(), (double *)out->val);
    HIPCHECK(hipStreamSynchronize(ctx->stream));
    if (info) {
        info->s_lo = info->lo = r.lo;
        info->s_hi = info->hi = r.hi;
        info->n_pl = info->n_pl_s = r.n_pl;
        info->passes = 1;
        info->reexpansions = r.reexp;
        info->penalty = info->s_penalty = r.penalty;
        info->s_check_terms = r.check_terms;
        info->chain_steps = r.products;
        info->ms_total = now_ms() - t0;
        info->ms_chain_kernel = r.kernel_ms;
        info->kernel_variant = r.variant;
    }
}

static void eigs_in_interval(chess_ctx *ctx, const chess_matrix *H, const chess_matrix *S,
                             double e_lo, double e_hi, const chess_pattern *pattern,
                             double *eig_out, int64_t capacity, int64_t *n_found,
                             chess_info *info, const chess_opts *opts) {
    const double t0 = now_ms();
    chess_opts o = resolve_opts(opts);
    check_matrix(H, "H");
    check_matrix(S, "S");
    if (!n_found) CHESS_THROW(CHESS_E_ARG, "n_found is null");
    if (capacity > 0 && !eig_out) CHESS_THROW(CHESS_E_ARG, "eig_out is null");
    if (!(e_hi > e_lo)) CHESS_THROW(CHESS_E_ARG, "empty interval");
    const Pattern *PH = get_pattern(ctx, &H->pat, "H pattern");
    const Pattern *PS = get_pattern(ctx, &S->pat, "S pattern");
    const Pattern *PK = get_pattern(ctx, pattern, "chain pattern");
    get_embed(ctx, PH, PK, "H in the chain pattern");
    get_embed(ctx, PS, PK, "S in the chain pattern");
    Frame F;
    build_frame(ctx, PH, (const double *)H->val, PS, (const double *)S->val, PK, o, F);
    double lo, hi;
    h_bounds(ctx, PH, F.Hp.as<double>(), o, &lo, &hi);
    const int b = PK->b;
    DevBuf Ht(sizeof(double) * (size_t)PH->nnzb * b * b);
    std::vector<double> mom;
    int n_pl = 0, reexp = 0, variant = -1;
    double kernel_ms = 0, penalty = std::numeric_limits<double>::quiet_NaN();
    for (int attempt = 0;; ++attempt) {
        double sigma, tau;
        hostmath::scale_shift(lo, hi, &sigma, &tau);
        n_pl = o.n_pl;
        if (n_pl <= 0) {
            n_pl = hostmath::degree(occupation(CHESS_ERFC, tau, o.eig_width), lo, hi, o.tol_fit, 8, 20000);
            if (n_pl < 0) CHESS_THROW(CHESS_E_NOCONV, "no degree up to 20000 reaches tol_fit %g", o.tol_fit);
        }
        HIPCHECK(launch_scale_shift(b, PH->nnzb, PH->d_brow.as<int32_t>(), PH->d_ci.as<int32_t>(), F.Hp.as<double>(), Ht.as<double>(), sigma, tau, ctx->stream));
        ChainRequest rq;
        rq.label = "eigenvalue chain";
        rq.PM = PH;
        rq.Mt = Ht.as<double>();
        rq.PK = PK;
        rq.n_pl = n_pl;
        rq.dtype = storage_dtype(o.precision);
        rq.opmode = operand_mode(o.precision);
        rq.moments = &mom;
        run_chain(ctx, rq);
        kernel_ms += rq.kernel_ms;
        variant = rq.variant;
        const hostmath::BoundsCheck chk = hostmath::bounds_check(mom, PK->n());
        penalty = chk.penalty;
        if (chk.ok) break;
        if (attempt >= o.max_reexpand) CHESS_THROW(CHESS_E_BOUNDS, "bounds [%g, %g] still fail after %d widenings", lo, hi, attempt);
        hostmath::widen(chk.side, &lo, &hi);
        reexp++;
    }
    hostmath::CountFunction N;
    N.init(mom, lo, hi, o.eig_width, 0);
    std::vector<double> ev = hostmath::eigenvalues(N, e_lo, e_hi, 1e-10);
    *n_found = (int64_t)ev.size();
    if ((int64_t)ev.size() > capacity)
        CHESS_THROW(CHESS_E_CAPACITY, "%lld eigenvalues in the interval, capacity %lld", (long long)ev.size(), (long long)capacity);
    std::copy(ev.begin(), ev.end(), eig_out);
    if (info) {
        info->lo = lo;
        info->hi = hi;
        info->s_lo = F.s.lo;
        info->s_hi = F.s.hi;
        info->n_pl = n_pl;
        info->n_pl_s = F.s.n_pl;
        info->passes = 1 + reexp;
        info->reexpansions = reexp;
        info->penalty = penalty;
        info->s_penalty = F.s.penalty;
        info->s_check_terms = F.s.check_terms;
        info->ms_total = now_ms() - t0;
        info->ms_chain_kernel = kernel_ms;
        info->kernel_variant = variant;
    }
}

static void chebyshev(chess_ctx *ctx, const chess_matrix *M, double lo, double hi,
                      const chess_pattern *pattern, int32_t n_pl, int32_t nq, const double *coef,
                      chess_matrix *acc_out, double *moments, const chess_opts *opts) {
    chess_opts o = resolve_opts(opts);
    check_matrix(M, "M");
    if (n_pl < 1) CHESS_THROW(CHESS_E_ARG, "n_pl must be >= 1");
    if (nq < 0 || nq > 4) CHESS_THROW(CHESS_E_ARG, "nq must be in 0..4");
    if (nq > 0 && (!coef || !acc_out)) CHESS_THROW(CHESS_E_ARG, "coefficients or outputs missing");
    if (!(hi > lo)) CHESS_THROW(CHESS_E_ARG, "empty interval");
    const Pattern *PM = get_pattern(ctx, &M->pat, "M pattern");
    const Pattern *PK = get_pattern(ctx, pattern, "chain pattern");
    if (PM->nb != PK->nb || PM->b != PK->b) CHESS_THROW(CHESS_E_ARG, "M and the pattern differ in size");
    for (int q = 0; q < nq; ++q) {
        check_matrix(&acc_out[q], "acc_out");
        require_same(get_pattern(ctx, &acc_out[q].pat, "acc_out pattern"), PK, "acc_out");
    }
    get_embed(ctx, PM, PK, "M in the chain pattern");
    hipStream_t st = ctx->stream;
    const int b = PK->b;
    DevBuf Mt(sizeof(double) * (size_t)PM->nnzb * b * b);
    double sigma, tau;
    hostmath::scale_shift(lo, hi, &sigma, &tau);
    HIPCHECK(launch_scale_shift(b, PM->nnzb, PM->d_brow.as<int32_t>(), PM->d_ci.as<int32_t>(), (const double *)M->val, Mt.as<double>(), sigma, tau, st));
    std::vector<std::unique_ptr<DevBuf>> accs;
    ChainRequest rq;
    rq.label = "chebyshev chain";
    rq.PM = PM;
    rq.Mt = Mt.as<double>();
    rq.PK = PK;
    rq.n_pl = n_pl;
    rq.nq = nq;
    rq.coef = coef;
    rq.dtype = storage_dtype(o.precision);
    rq.opmode = operand_mode(o.precision);
    for (int q = 0; q < nq; ++q) {
        accs.push_back(std::make_unique<DevBuf>(sizeof(double) * (size_t)PK->nnzb * b * b));
        rq.acc[q] = accs.back()->as<double>();
    }
    std::vector<double> mom;
    rq.moments = &mom;
    run_chain(ctx, rq);
    for (int q = 0; q < nq; ++q) transpose_into(ctx, PK, rq.acc[q], (double *)acc_out[q].val);
    HIPCHECK(hipStreamSynchronize(st));
    if (moments) std::copy(mom.begin(), mom.end(), moments);
}

static void masked_product_api(chess_ctx *ctx, const chess_matrix *A, const chess_matrix *B,
                               chess_matrix *C) {
    check_matrix(A, "A");
    check_matrix(B, "B");
    check_matrix(C, "C");
    const Pattern *PA = get_pattern(ctx, &A->pat, "A pattern");
    const Pattern *PB = get_pattern(ctx, &B->pat, "B pattern");
    const Pattern *PC = get_pattern(ctx, &C->pat, "C pattern");
    if (PA->nb != PB->nb || PA->nb != PC->nb || PA->b != PB->b || PA->b != PC->b)
        CHESS_THROW(CHESS_E_ARG, "A, B, C differ in size or block edge");
    DevBuf BT(sizeof(double) * (size_t)PB->nnzb * PB->b * PB->b);
    transpose_into(ctx, PB, (const double *)B->val, BT.as<double>());
    product(ctx, 0, get_plan(ctx, PA, PB, PC, 0), A->val, BT.p, C->val, Epilogue{});
    HIPCHECK(hipStreamSynchronize(ctx->stream));
}

// ---------------------------------------------------------------------------
// batches of independent systems
// ---------------------------------------------------------------------------

// Block-diagonal concatenation of patterns (all with block edge b).
static const Pattern *concat_patterns(chess_ctx *ctx, const std::vector<const Pattern *> &ps,
                                      const char *what) {
    const int b = ps[0]->b;
    int nb = 0;
    int64_t nnzb = 0;
    for (const Pattern *p : ps) {
        nb += p->nb;
        nnzb += p->nnzb;
    }
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    rp.reserve((size_t)nb + 1);
    ci.reserve((size_t)nnzb);
    rp.push_back(0);
    int r0 = 0;
    int64_t z0 = 0;
    for (const Pattern *p : ps) {
        for (int i = 0; i < p->nb; ++i) rp.push_back(z0 + p->rp[i + 1]);
        for (int32_t c : p->ci) ci.push_back(c + r0);
        r0 += p->nb;
        z0 += p->nnzb;
    }
    return get_pattern_host(ctx, b, nb, nnzb, std::move(rp), std::move(ci), what);
}

// One group of systems with the same block edge: every step of the
// single-system method, with the chains and the sandwich products run once
// over the block-diagonal concatenation.
static void batched_group(chess_ctx *ctx, const std::vector<int> &idx, const chess_batch_item *items,
                          const chess_opts &o, bool use_graph, double *ms_chains) {
    hipStream_t st = ctx->stream;
    const int nsys = (int)idx.size();
    const int dtype = storage_dtype(o.precision);
    std::vector<const Pattern *> PHs, PSs, PKs;
    for (int i : idx) {
        const chess_batch_item &it = items[i];
        const Pattern *PH = get_pattern(ctx, &it.H->pat, "H pattern");
        const Pattern *PS = get_pattern(ctx, &it.S->pat, "S pattern");
        const Pattern *PK = get_pattern(ctx, it.pattern, "kernel pattern");
        if (PH->nb != PK->nb || PS->nb != PK->nb || PH->b != PK->b || PS->b != PK->b)
            CHESS_THROW(CHESS_E_ARG, "system %d: H, S and the pattern differ in size or block edge", i);
        get_embed(ctx, PH, PK, "H in the kernel pattern");
        get_embed(ctx, PS, PK, "S in the kernel pattern");
        for (int q = 0; q < 3; ++q)
            if (it.K_out[q]) {
                check_matrix(it.K_out[q], "K_out");
                require_same(get_pattern(ctx, &it.K_out[q]->pat, "K_out pattern"), PK, "K_out");
            }
        if (it.Sinvhalf_out) require_same(get_pattern(ctx, &it.Sinvhalf_out->pat, "Sinvhalf_out pattern"), PK, "Sinvhalf_out");
        if (it.Sinv_out) require_same(get_pattern(ctx, &it.Sinv_out->pat, "Sinv_out pattern"), PK, "Sinv_out");
        PHs.push_back(PH);
        PSs.push_back(PS);
        PKs.push_back(PK);
    }
    const int b = PKs[0]->b;
    const int64_t bb = (int64_t)b * b;
    const Pattern *PH = concat_patterns(ctx, PHs, "batched H pattern");
    const Pattern *PS = concat_patterns(ctx, PSs, "batched S pattern");
    const Pattern *PK = concat_patterns(ctx, PKs, "batched kernel pattern");
    std::vector<int32_t> row0(nsys + 1, 0), row_sys((size_t)PK->nb);
    std::vector<int64_t> offH(nsys + 1, 0), offS(nsys + 1, 0), offK(nsys + 1, 0);
    for (int s = 0; s < nsys; ++s) {
        row0[s + 1] = row0[s] + PKs[s]->nb;
        offH[s + 1] = offH[s] + PHs[s]->nnzb;
        offS[s + 1] = offS[s] + PSs[s]->nnzb;
        offK[s + 1] = offK[s] + PKs[s]->nnzb;
        for (int r = row0[s]; r < row0[s + 1]; ++r) row_sys[r] = s;
    }
    DevBuf d_row_sys;
    upload(d_row_sys, row_sys, st);
    DevBuf Hs(sizeof(double) * (size_t)PH->nnzb * bb), Ss(sizeof(double) * (size_t)PS->nnzb * bb);
    for (int s = 0; s < nsys; ++s) {
        const chess_batch_item &it = items[idx[s]];
        HIPCHECK(hipMemcpyAsync(Hs.as<double>() + offH[s] * bb, it.H->val, sizeof(double) * PHs[s]->nnzb * bb, hipMemcpyDeviceToDevice, st));
        HIPCHECK(hipMemcpyAsync(Ss.as<double>() + offS[s] * bb, it.S->val, sizeof(double) * PSs[s]->nnzb * bb, hipMemcpyDeviceToDevice, st));
    }
    // S bounds per system, then one S chain for x^-1/2 and x^-1
    std::vector<double> slo(nsys), shi(nsys), ssig(nsys), stau(nsys);
    std::vector<int> npls(nsys);
    int npls_max = 2;
    DevBuf dsig(sizeof(double) * nsys), dtau(sizeof(double) * nsys);
    DevBuf St(Ss.bytes);
    auto scale_all = [&]() {
        for (int s = 0; s < nsys; ++s) hostmath::scale_shift(slo[s], shi[s], &ssig[s], &stau[s]);
        HIPCHECK(hipMemcpyAsync(dsig.p, ssig.data(), sizeof(double) * nsys, hipMemcpyHostToDevice, st));
        HIPCHECK(hipMemcpyAsync(dtau.p, stau.data(), sizeof(double) * nsys, hipMemcpyHostToDevice, st));
        HIPCHECK(launch_scale_shift_rows(b, PS->nnzb, PS->d_brow.as<int32_t>(), PS->d_ci.as<int32_t>(),
                                         d_row_sys.as<int32_t>(), dsig.as<double>(), dtau.as<double>(),
                                         Ss.as<double>(), St.as<double>(), st));
        // the host vectors are rewritten by the next widening
        HIPCHECK(hipStreamSynchronize(st));
    };
    for (int s = 0; s < nsys; ++s)
        s_bounds(ctx, PSs[s], (const double *)items[idx[s]].S->val, o, true, &slo[s], &shi[s]);
    // the intervals the predictor's features describe S with (before any widening)
    const std::vector<double> slo0 = slo, shi0 = shi;
    // Eq. 6 and the growth test on every system's S, as in single calls: one
    // moments-only chain over the batch, each system running the
    // penalty_degree(n) terms Eq. 6 needs on its rows; failing systems widen
    // (the matrix-power rule) and the check runs again
    std::vector<double> spen(nsys, NAN);
    std::vector<int> sre(nsys, 0), nchk(nsys);
    int nchk_max = 2, check_products = 0;
    for (int s = 0; s < nsys; ++s) {
        nchk[s] = hostmath::penalty_degree(PKs[s]->n());
        nchk_max = std::max(nchk_max, nchk[s]);
    }
    for (int attempt = 0;; ++attempt) {
        scale_all();
        std::vector<double> cmom;
        BatchChain cc;
        cc.PM = PS;
        cc.PK = PK;
        cc.Mt = St.as<double>();
        cc.n_pl = nchk_max;
        cc.nq = 0;
        cc.dtype = dtype;
        cc.opmode = 0;  // the storage precision's operands, as in power_chain
        cc.row0 = &row0;
        cc.d_row_sys = d_row_sys.as<int32_t>();
        cc.sys_npl = &nchk;
        cc.use_graph = use_graph;
        cc.moments = &cmom;
        run_chain_batched(ctx, cc);
        check_products += std::max(nchk_max - 2, 0);
        bool all_ok = true;
        for (int s = 0; s < nsys; ++s) {
            std::vector<double> t(nchk[s]);
            for (int k = 0; k < nchk[s]; ++k) t[k] = cmom[(size_t)k * nsys + s];
            const hostmath::BoundsCheck chk = hostmath::bounds_check(t, PKs[s]->n());
            spen[s] = chk.penalty;
            if (chk.ok) continue;
            if (attempt >= o.max_reexpand)
                CHESS_THROW(CHESS_E_BOUNDS, "system %d: bounds of S [%g, %g] still fail after %d widenings", idx[s],
                            slo[s], shi[s], attempt);
            widen_power(chk, &slo[s], &shi[s]);
            sre[s]++;
            all_ok = false;
        }
        if (all_ok) break;
    }
    for (int s = 0; s < nsys; ++s) {
        int m = o.n_pl_s;
        if (m <= 0) {
            m = 1;
            for (double a : {-0.5, -1.0}) {
                const int d = hostmath::degree([a](double x) { return std::pow(x, a); }, slo[s], shi[s], o.tol_fit_s, 8, 20000);
                if (d < 0) CHESS_THROW(CHESS_E_NOCONV, "system %d: no degree reaches tol_fit_s", idx[s]);
                m = std::max(m, d);
            }
        }
        npls[s] = m;
        npls_max = std::max(npls_max, m);
    }
    auto coef_table = [&](int nq, int n_pl, const std::vector<int> &own, auto &&fn) {
        std::vector<double> tab((size_t)nq * n_pl * nsys, 0.0);
        for (int s = 0; s < nsys; ++s)
            for (int q = 0; q < nq; ++q) {
                const std::vector<double> c = fn(s, q, own[s]);
                for (int k = 0; k < own[s]; ++k) tab[((size_t)q * n_pl + k) * nsys + s] = c[k];
            }
        return tab;
    };
    const std::vector<double> stab = coef_table(2, npls_max, npls, [&](int s, int q, int m) {
        const double a = q == 0 ? -0.5 : -1.0;
        return hostmath::cheb_coeffs([a](double x) { return std::pow(x, a); }, slo[s], shi[s], m);
    });
    const size_t kbytes = sizeof(double) * (size_t)PK->nnzb * bb;
    Frame F;
    F.accX.alloc(kbytes);
    DevBuf accSinv(kbytes);
    std::vector<double> smom;
    BatchChain sc;
    sc.PM = PS;
    sc.PK = PK;
    sc.Mt = St.as<double>();
    sc.n_pl = npls_max;
    sc.nq = 2;
    sc.dtype = dtype;
    sc.opmode = operand_mode(o.precision);
    sc.coef_tab = stab.data();
    sc.acc[0] = F.accX.as<double>();
    sc.acc[1] = accSinv.as<double>();
    sc.row0 = &row0;
    sc.d_row_sys = d_row_sys.as<int32_t>();
    sc.sys_npl = &npls;
    sc.use_graph = use_graph;
    sc.moments = &smom;
    run_chain_batched(ctx, sc);
    St.release();
    for (int s = 0; s < nsys; ++s) {
        std::vector<double> t(npls[s]);
        for (int k = 0; k < npls[s]; ++k) t[k] = smom[(size_t)k * nsys + s];
        if (!growth_ok(t, PKs[s]->n())) CHESS_THROW(CHESS_E_BOUNDS, "system %d: bounds of S fail the growth test", idx[s]);
    }
    // H' = sym(P_H o (X P_K o (H X))) over the whole batch
    {
        DevBuf ZT(kbytes);
        product(ctx, 0, get_plan(ctx, PK, PH, PK, 0), F.accX.p, Hs.p, ZT.p, Epilogue{});
        F.X.alloc(kbytes);
        transpose_into(ctx, PK, F.accX.as<double>(), F.X.as<double>());
        DevBuf Hraw(Hs.bytes);
        product(ctx, 0, get_plan(ctx, PK, PK, PH, 0), F.X.p, ZT.p, Hraw.p, Epilogue{});
        F.Hp.alloc(Hs.bytes);
        HIPCHECK(launch_symmetrize(b, PH->nnzb, PH->d_tmap.as<int64_t>(), Hraw.as<double>(), F.Hp.as<double>(), st));
    }
    // bounds, degree and trial mu per system
    std::vector<double> lo(nsys), hi(nsys), hsig(nsys), htau(nsys), kTs(nsys), nes(nsys);
    std::vector<std::array<double, 3>> mus(nsys), preds(nsys);
    std::vector<int> npl(nsys);
    int npl_max = 2;
    const double nan = std::numeric_limits<double>::quiet_NaN();
    for (int s = 0; s < nsys; ++s) {
        const chess_batch_item &it = items[idx[s]];
        const double *Hp = F.Hp.as<double>() + offH[s] * bb;
        kTs[s] = it.kT;
        nes[s] = it.n_electrons;
        preds[s] = {nan, nan, nan};
        double mu_half = 0.0;
        if (!(std::isfinite(o.bounds[0]) && std::isfinite(o.bounds[1])) &&
            (o.bounds_mode == CHESS_BOUNDS_LEARNED || o.bounds_mode == CHESS_BOUNDS_LEARNED_LANCZOS)) {
            Features fe;
            compute_features(ctx, PHs[s], Hp, PKs[s], slo0[s], shi0[s], it.n_electrons, it.kT, fe);
            double pr[3];
            predict(ctx, fe, pr);
            const double w = 0.5 * (fe.g_hi - fe.g_lo);
            lo[s] = std::max(fe.g_lo, pr[0] - ctx->model.margin_lo * w);
            hi[s] = std::min(fe.g_hi, pr[1] + ctx->model.margin_hi * w);
            if (o.bounds_mode == CHESS_BOUNDS_LEARNED_LANCZOS) {
                chess_opts ol = o;
                ol.bounds_mode = CHESS_BOUNDS_LANCZOS;
                double llo, lhi;
                h_bounds(ctx, PHs[s], Hp, ol, &llo, &lhi);
                lo[s] = std::max(lo[s], llo);
                hi[s] = std::min(hi[s], lhi);
            }
            if (!(hi[s] > lo[s])) {
                lo[s] = fe.g_lo;
                hi[s] = fe.g_hi;
            }
            preds[s] = {pr[0], pr[1], pr[2]};
            mu_half = ctx->model.mu_half * w;
        } else {
            h_bounds(ctx, PHs[s], Hp, o, &lo[s], &hi[s]);
        }
        for (int q = 0; q < 3; ++q) {
            double m = it.mu_trial[q];
            if (!std::isfinite(m)) {
                if (!std::isfinite(preds[s][2]))
                    CHESS_THROW(CHESS_E_ARG, "system %d: mu_trial[%d] not given and no prediction (learned bounds modes)", idx[s], q);
                m = preds[s][2] + (q - 1) * mu_half;
            }
            mus[s][q] = m;
        }
        hostmath::scale_shift(lo[s], hi[s], &hsig[s], &htau[s]);
        int m = o.n_pl;
        if (m <= 0) {
            m = hostmath::degree(occupation(o.smearing, htau[s], it.kT), lo[s], hi[s], o.tol_fit, 8, 20000);
            if (m < 0) CHESS_THROW(CHESS_E_NOCONV, "system %d: no degree up to 20000 reaches tol_fit", idx[s]);
        }
        npl[s] = m;
        npl_max = std::max(npl_max, m);
    }
    HIPCHECK(hipMemcpyAsync(dsig.p, hsig.data(), sizeof(double) * nsys, hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(dtau.p, htau.data(), sizeof(double) * nsys, hipMemcpyHostToDevice, st));
    DevBuf Ht(Hs.bytes);
    HIPCHECK(launch_scale_shift_rows(b, PH->nnzb, PH->d_brow.as<int32_t>(), PH->d_ci.as<int32_t>(), d_row_sys.as<int32_t>(),
                                     dsig.as<double>(), dtau.as<double>(), F.Hp.as<double>(), Ht.as<double>(), st));
    const std::vector<double> htab = coef_table(3, npl_max, npl, [&](int s, int q, int m) {
        return hostmath::cheb_coeffs(occupation(o.smearing, mus[s][q], kTs[s]), lo[s], hi[s], m);
    });
    DevBuf accK[3];
    for (auto &a : accK) a.alloc(kbytes);
    std::vector<double> hmom;
    BatchChain hc;
    hc.PM = PH;
    hc.PK = PK;
    hc.Mt = Ht.as<double>();
    hc.n_pl = npl_max;
    hc.nq = 3;
    hc.dtype = dtype;
    hc.opmode = operand_mode(o.precision);
    hc.coef_tab = htab.data();
    for (int q = 0; q < 3; ++q) hc.acc[q] = accK[q].as<double>();
    hc.row0 = &row0;
    hc.d_row_sys = d_row_sys.as<int32_t>();
    hc.sys_npl = &npl;
    hc.use_graph = use_graph;
    hc.moments = &hmom;
    run_chain_batched(ctx, hc);
    *ms_chains += sc.kernel_ms + hc.kernel_ms;
    Ht.release();
    // per system: Eq. 6 and growth checks, mu from the moments, N at the trial mu
    std::vector<double> mu_star(nsys), ne_tr(3 * (size_t)nsys), pen(nsys);
    std::vector<double> homo_s(nsys, nan), lumo_s(nsys, nan);
    std::vector<int> iters(nsys);
    std::vector<char> failed(nsys, 0);
    std::vector<int> failed_pos;
    for (int s = 0; s < nsys; ++s) {
        std::vector<double> t(npl[s]);
        for (int k = 0; k < npl[s]; ++k) t[k] = hmom[(size_t)k * nsys + s];
        const hostmath::BoundsCheck chk = hostmath::bounds_check(t, PKs[s]->n());
        pen[s] = chk.penalty;
        if (!chk.ok) {
            // rejected bounds: this system is redone below with the
            // Gershgorin interval (unless that is what failed)
            const bool rigorous = o.bounds_mode == CHESS_BOUNDS_GERSHGORIN &&
                                  !(std::isfinite(o.bounds[0]) && std::isfinite(o.bounds[1]));
            if (rigorous)
                CHESS_THROW(CHESS_E_BOUNDS, "system %d: Gershgorin bounds [%g, %g] fail Eq. 6 or the growth test", idx[s], lo[s], hi[s]);
            failed[s] = 1;
            failed_pos.push_back(s);
            continue;
        }
        hostmath::CountFunction N;
        N.init(t, lo[s], hi[s], kTs[s], o.smearing == CHESS_ERFC ? 0 : 1);
        const double tol_ne = o.tol_ne > 0 ? o.tol_ne : 1e-8 * nes[s];
        double m = nan;
        int itn = 0;
        if (!hostmath::bisect_mu(N, nes[s], tol_ne, lo[s] - 20 * kTs[s], hi[s] + 20 * kTs[s], &m, &itn))
            CHESS_THROW(CHESS_E_NOCONV, "system %d: N(mu) does not bracket %g electrons", idx[s], nes[s]);
        mu_star[s] = m;
        iters[s] = itn;
        homo_lumo(N, nes[s], (double)PKs[s]->n(), lo[s], hi[s], kTs[s], &homo_s[s], &lumo_s[s]);
        for (int q = 0; q < 3; ++q) ne_tr[3 * (size_t)s + q] = N(mus[s][q]);
    }
    // K at the trial mu: K = P_K o (X P_K o (K' X)) over the batch, then per system
    DevBuf Kb(kbytes);
    const int nparts = 256;
    DevBuf part(sizeof(double) * (nparts + 1));
    for (int q = 0; q < 3; ++q) {
        bool any = false;
        for (int s = 0; s < nsys; ++s) any = any || items[idx[s]].K_out[q];
        if (!any) continue;
        post_transform(ctx, PK, F, accK[q].as<double>(), PS, Ss.as<double>(), Kb.as<double>());
        for (int s = 0; s < nsys; ++s) {
            chess_matrix *Ko = items[idx[s]].K_out[q];
            if (!Ko || failed[s]) continue;
            HIPCHECK(hipMemcpyAsync(Ko->val, Kb.as<double>() + offK[s] * bb, sizeof(double) * PKs[s]->nnzb * bb, hipMemcpyDeviceToDevice, st));
            if (q == 1 && items[idx[s]].info) {
                const EmbedMap *es = get_embed(ctx, PSs[s], PKs[s], "S in the kernel pattern");
                HIPCHECK(launch_trace_product(b, PSs[s]->nnzb, es->d_map_t.as<int64_t>(), (const double *)Ko->val,
                                              (const double *)items[idx[s]].S->val, part.as<double>(), nparts, st));
                HIPCHECK(launch_reduce_rows(1, nparts, part.as<double>(), part.as<double>() + nparts, st));
                double tr = 0.0;
                HIPCHECK(hipMemcpyAsync(&tr, part.as<double>() + nparts, sizeof(double), hipMemcpyDeviceToHost, st));
                HIPCHECK(hipStreamSynchronize(st));
                items[idx[s]].info->tr_ks = tr;
            }
        }
    }
    // S^-1/2 = X and S^-1 (the accumulators hold the transposes)
    DevBuf Sinv(kbytes);
    transpose_into(ctx, PK, accSinv.as<double>(), Sinv.as<double>());
    for (int s = 0; s < nsys; ++s) {
        if (failed[s]) continue;
        const chess_batch_item &it = items[idx[s]];
        const size_t bytes = sizeof(double) * PKs[s]->nnzb * bb;
        if (it.Sinvhalf_out) HIPCHECK(hipMemcpyAsync(it.Sinvhalf_out->val, F.X.as<double>() + offK[s] * bb, bytes, hipMemcpyDeviceToDevice, st));
        if (it.Sinv_out) HIPCHECK(hipMemcpyAsync(it.Sinv_out->val, Sinv.as<double>() + offK[s] * bb, bytes, hipMemcpyDeviceToDevice, st));
        if (it.ne_trial)
            for (int q = 0; q < 3; ++q) it.ne_trial[q] = ne_tr[3 * (size_t)s + q];
        if (chess_info *info = it.info) {
            info->mu = mu_star[s];
            info->lo = lo[s];
            info->hi = hi[s];
            info->s_lo = slo[s];
            info->s_hi = shi[s];
            info->ne_chain = ne_tr[3 * (size_t)s + 1];
            info->penalty = pen[s];
            info->n_pl = npl[s];
            info->n_pl_s = npls[s];
            info->passes = 1;
            info->bisect_iters = iters[s];
            info->chain_steps = std::max(npl_max - 2, 0) + std::max(npls_max - 2, 0) + check_products;
            info->reexpansions = sre[s];
            info->s_penalty = spen[s];
            info->s_check_terms = nchk[s];
            info->kernel_variant = hc.variant;
            info->pred_lo = preds[s][0];
            info->pred_hi = preds[s][1];
            info->pred_mu = preds[s][2];
            info->homo = homo_s[s];
            info->lumo = lumo_s[s];
        }
    }
    HIPCHECK(hipStreamSynchronize(st));
    if (!failed_pos.empty()) {
        // the rejected systems again, as a batch of their own, with the
        // rigorous Gershgorin interval and the trial mu of the first attempt
        std::vector<chess_batch_item> sub;
        for (int s : failed_pos) {
            chess_batch_item it = items[idx[s]];
            for (int q = 0; q < 3; ++q) it.mu_trial[q] = mus[s][q];
            sub.push_back(it);
        }
        chess_opts o2 = o;
        o2.bounds_mode = CHESS_BOUNDS_GERSHGORIN;
        o2.bounds[0] = o2.bounds[1] = nan;
        std::vector<int> sidx(sub.size());
        for (size_t k = 0; k < sub.size(); ++k) sidx[k] = (int)k;
        batched_group(ctx, sidx, sub.data(), o2, use_graph, ms_chains);
        for (int s : failed_pos)
            if (chess_info *info = items[idx[s]].info) {
                info->fallback |= 1;
                info->reexpansions += 1;
                info->pred_lo = preds[s][0];
                info->pred_hi = preds[s][1];
                info->pred_mu = preds[s][2];
            }
    }
}

static void fermi_batched(chess_ctx *ctx, int32_t nsys, const chess_batch_item *items,
                          const chess_opts *opts) {
    const double t0 = now_ms();
    chess_opts o = resolve_opts(opts);
    if (nsys <= 0 || !items) CHESS_THROW(CHESS_E_ARG, "empty batch");
    std::vector<int> by4, by9;
    for (int i = 0; i < nsys; ++i) {
        const chess_batch_item &it = items[i];
        check_matrix(it.H, "H");
        check_matrix(it.S, "S");
        if (!it.pattern) CHESS_THROW(CHESS_E_ARG, "system %d: null pattern", i);
        if (!(it.kT > 0)) CHESS_THROW(CHESS_E_ARG, "system %d: kT must be positive", i);
        fill_info_defaults(it.info);
        (it.pattern->b == 4 ? by4 : by9).push_back(i);
    }
    // CHESS_BATCH_GRAPH=0 in the environment runs the products without graph capture
    bool use_graph = true;
    if (const char *env = std::getenv("CHESS_BATCH_GRAPH")) use_graph = std::strcmp(env, "0") != 0;
    double ms_chains = 0.0;
    if (!by4.empty()) batched_group(ctx, by4, items, o, use_graph, &ms_chains);
    if (!by9.empty()) batched_group(ctx, by9, items, o, use_graph, &ms_chains);
    const double ms = now_ms() - t0;
    for (int i = 0; i < nsys; ++i)
        if (items[i].info) {
            items[i].info->ms_total = ms;
            items[i].info->ms_chain_kernel = ms_chains;
        }
}

// Features of the generalized problem (H, S) for the learned predictor: the
// orthogonal frame as in the Fermi operator, then compute_features.
static void features_api(chess_ctx *ctx, const chess_matrix *H, const chess_matrix *S,
                         const chess_pattern *pattern, double n_e, double kT, float *feat,
                         double *gersh, const chess_opts *opts) {
    chess_opts o = resolve_opts(opts);
    check_matrix(H, "H");
    check_matrix(S, "S");
    if (!feat) CHESS_THROW(CHESS_E_ARG, "null feature output");
    if (!(kT > 0)) CHESS_THROW(CHESS_E_ARG, "kT must be positive");
    const Pattern *PH = get_pattern(ctx, &H->pat, "H pattern");
    const Pattern *PS = get_pattern(ctx, &S->pat, "S pattern");
    const Pattern *PK = get_pattern(ctx, pattern, "kernel pattern");
    if (PH->nb != PK->nb || PS->nb != PK->nb || PH->b != PK->b || PS->b != PK->b)
        CHESS_THROW(CHESS_E_ARG, "H, S and the pattern differ in size or block edge");
    get_embed(ctx, PH, PK, "H in the kernel pattern");
    get_embed(ctx, PS, PK, "S in the kernel pattern");
    Frame F;
    build_frame(ctx, PH, (const double *)H->val, PS, (const double *)S->val, PK, o, F);
    Features fe;
    compute_features(ctx, PH, F.Hp.as<double>(), PK, F.s_lo0, F.s_hi0, n_e, kT, fe);
    std::memcpy(feat, fe.f, sizeof(fe.f));
    if (gersh) {
        gersh[0] = fe.g_lo;
        gersh[1] = fe.g_hi;
    }
}

static void model_load(chess_ctx *ctx, const float *blob, int64_t n) {
    if (!blob || n != CHESS_MODEL_FLOATS)
        CHESS_THROW(CHESS_E_ARG, "model blob must hold %d floats (got %lld)", CHESS_MODEL_FLOATS, (long long)n);
    for (int64_t k = 0; k < n; ++k)
        if (!std::isfinite(blob[k])) CHESS_THROW(CHESS_E_ARG, "model blob entry %lld is not finite", (long long)k);
    for (int k = 0; k < kMlpIn; ++k)
        if (!(blob[kMlpIn + k] > 0)) CHESS_THROW(CHESS_E_ARG, "model: inverse feature scale %d must be positive", k);
    Model &M = ctx->model;
    M.loaded = false;
    M.blob.assign(blob, blob + n);
    M.norm.alloc(sizeof(float) * kMlpNorm);
    M.params.alloc(sizeof(float) * kMlpParams);
    hipStream_t st = ctx->stream;
    HIPCHECK(hipMemcpyAsync(M.norm.p, blob, sizeof(float) * kMlpNorm, hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(M.params.p, blob + kMlpNorm + 3, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, st));
    HIPCHECK(hipStreamSynchronize(st));
    M.margin_lo = std::max(0.0f, blob[kMlpNorm]);
    M.margin_hi = std::max(0.0f, blob[kMlpNorm + 1]);
    M.mu_half = std::max(0.0f, blob[kMlpNorm + 2]);
    M.loaded = true;
}

template <typename F>
static int guarded(chess_ctx *ctx, F &&f) {
    if (!ctx) return CHESS_E_ARG;
    try {
        HIPCHECK(hipSetDevice(ctx->device));
        f();
        ctx->err = "no error";
        return CHESS_OK;
    } catch (const Error &e) {
        set_err(ctx, e);
        return e.code;
    } catch (const std::bad_alloc &) {
        ctx->err = "host allocation failed";
        return CHESS_E_OOM;
    } catch (...) {
        ctx->err = "unexpected exception";
        return CHESS_E_HIP;
    }
}

int ctx_device(const chess_ctx *ctx) { return ctx->device; }
hipStream_t ctx_stream(const chess_ctx *ctx) { return ctx->stream; }
void ctx_set_error(chess_ctx *ctx, const char *msg) { ctx->err = msg; }

}  // namespace chess

using chess::Error;

extern "C" {

int chess_degree(int32_t fn, double param, double lo, double hi, double tol_fit, int32_t *n_pl_out) {
    if (!n_pl_out || !(hi > lo) || !(tol_fit > 0) || !std::isfinite(lo) || !std::isfinite(hi))
        return CHESS_E_ARG;
    chess::hostmath::Fn f;
    if (fn == CHESS_FN_ERFC || fn == CHESS_FN_FERMI_DIRAC) {
        if (!(param > 0)) return CHESS_E_ARG;
        f = chess::occupation(fn == CHESS_FN_ERFC ? CHESS_ERFC : CHESS_FERMI_DIRAC, 0.5 * (lo + hi), param);
    } else if (fn == CHESS_FN_PENALTY) {
        if (!(param >= 1) || param > 9.0e18) return CHESS_E_ARG;
        try {
            *n_pl_out = chess::hostmath::penalty_degree((long long)param);
            return CHESS_OK;
        } catch (...) {
            return CHESS_E_OOM;
        }
    } else if (fn == CHESS_FN_POWER) {
        const bool whole = param >= 0 && std::floor(param) == param;
        if (!whole && !(lo > 0)) return CHESS_E_ARG;
        const double a = param;
        f = [a](double x) { return std::pow(x, a); };
    } else {
        return CHESS_E_ARG;
    }
    try {
        const int m = chess::hostmath::degree(f, lo, hi, tol_fit, 8, 20000);
        if (m < 0) return CHESS_E_NOCONV;
        *n_pl_out = m;
        return CHESS_OK;
    } catch (...) {
        return CHESS_E_OOM;
    }
}

void chess_default_opts(chess_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    const double nan = std::numeric_limits<double>::quiet_NaN();
    o->precision = CHESS_F32;
    o->smearing = CHESS_ERFC;
    o->bounds_mode = CHESS_BOUNDS_GERSHGORIN;
    o->n_pl = 0;
    o->n_pl_s = 0;
    o->store_history = 0;
    o->max_reexpand = 3;
    o->lanczos_steps = 40;
    o->tol_fit = 0;
    o->tol_fit_s = 0;
    o->tol_ne = 0;
    o->bounds[0] = o->bounds[1] = nan;
    o->s_bounds[0] = o->s_bounds[1] = nan;
    o->mu = nan;
    o->mu_bracket[0] = o->mu_bracket[1] = nan;
    o->eig_width = 1e-3;
    o->bound_margin = 0.02;
    o->adapt_kt = 0;
    o->max_kt_halvings = 4;
    o->kt_ratio = 1.25;
    o->tol_energy = 0;
    o->sinvhalf_in = nullptr;
    o->sinvhalf_out = nullptr;
}

int chess_create(chess_ctx **out, int device, void *stream) {
    if (!out) return CHESS_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CHESS_E_HIP;
    if (hipSetDevice(device) != hipSuccess) return CHESS_E_HIP;
    // the fixed workspace of chess_mlp_grad_noalloc: its address on this device
    if (chess::noalloc_scratch_init(device) != hipSuccess) return CHESS_E_HIP;
    chess_ctx *c = new (std::nothrow) chess_ctx();
    if (!c) return CHESS_E_OOM;
    c->device = device;
    c->stream = (hipStream_t)stream;
    *out = c;
    return CHESS_OK;
}

int chess_destroy(chess_ctx *ctx) {
    if (!ctx) return CHESS_E_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    delete ctx;
    return CHESS_OK;
}

int chess_set_progress(chess_ctx *ctx, chess_progress_fn fn, void *user, int32_t every) {
    if (!ctx) return CHESS_E_ARG;
    if (fn && every <= 0) {
        ctx->err = "chess_set_progress: every must be positive";
        return CHESS_E_ARG;
    }
    ctx->progress = fn;
    ctx->progress_user = user;
    ctx->progress_every = fn ? every : 0;
    return CHESS_OK;
}

const char *chess_last_error(const chess_ctx *ctx) {
    if (!ctx) return "null context";
    return ctx->err.c_str();
}

int chess_fermi_operator(chess_ctx *ctx, const chess_matrix *H, const chess_matrix *S,
                         const chess_pattern *pattern, double n_electrons, double kT,
                         chess_matrix *K_out, chess_info *info, const chess_opts *opts) {
    chess::fill_info_defaults(info);
    return chess::guarded(ctx, [&] { chess::fermi_operator(ctx, H, S, pattern, n_electrons, kT, K_out, info, opts); });
}

int chess_matrix_power(chess_ctx *ctx, const chess_matrix *S, double a,
                       const chess_pattern *pattern, chess_matrix *Sa_out, chess_info *info,
                       const chess_opts *opts) {
    chess::fill_info_defaults(info);
    return chess::guarded(ctx, [&] { chess::matrix_power(ctx, S, a, pattern, Sa_out, info, opts); });
}

int chess_eigs_in_interval(chess_ctx *ctx, const chess_matrix *H, const chess_matrix *S,
                           double lo, double hi, const chess_pattern *pattern, double *eig_out,
                           int64_t capacity, int64_t *n_found, chess_info *info,
                           const chess_opts *opts) {
    chess::fill_info_defaults(info);
    return chess::guarded(ctx, [&] {
        chess::eigs_in_interval(ctx, H, S, lo, hi, pattern, eig_out, capacity, n_found, info, opts);
    });
}

int chess_chebyshev(chess_ctx *ctx, const chess_matrix *M, double lo, double hi,
                    const chess_pattern *pattern, int32_t n_pl, int32_t nq, const double *coef,
                    chess_matrix *acc_out, double *moments, const chess_opts *opts) {
    return chess::guarded(ctx, [&] { chess::chebyshev(ctx, M, lo, hi, pattern, n_pl, nq, coef, acc_out, moments, opts); });
}

int chess_masked_product(chess_ctx *ctx, const chess_matrix *A, const chess_matrix *B,
                         chess_matrix *C) {
    return chess::guarded(ctx, [&] { chess::masked_product_api(ctx, A, B, C); });
}

int chess_fermi_operator_batched(chess_ctx *ctx, int32_t nsys, const chess_batch_item *items,
                                 const chess_opts *opts) {
    return chess::guarded(ctx, [&] { chess::fermi_batched(ctx, nsys, items, opts); });
}

int chess_features(chess_ctx *ctx, const chess_matrix *H, const chess_matrix *S,
                   const chess_pattern *pattern, double n_electrons, double kT, float *feat_out,
                   double *gersh_out, const chess_opts *opts) {
    return chess::guarded(ctx, [&] { chess::features_api(ctx, H, S, pattern, n_electrons, kT, feat_out, gersh_out, opts); });
}

int chess_mlp_forward(chess_ctx *ctx, const float *params, const float *norm, const float *x,
                      int32_t batch, float *hidden, float *y) {
    return chess::guarded(ctx, [&] {
        if (!params || !x || !y || batch < 0) CHESS_THROW(CHESS_E_ARG, "mlp_forward: null pointer or negative batch");
        HIPCHECK(chess::launch_mlp_forward(params, norm, x, batch, hidden, y, ctx->stream));
    });
}

int chess_mlp_grad(chess_ctx *ctx, const float *params, const float *x, const float *hidden,
                   const float *y, const float *target, int32_t batch, float *work, float *grad,
                   double *loss) {
    return chess::guarded(ctx, [&] {
        if (!params || !x || !hidden || !y || !target || !work || !grad || batch <= 0)
            CHESS_THROW(CHESS_E_ARG, "mlp_grad: null pointer or empty batch");
        double *dl = nullptr;
        if (loss) {
            if (!ctx->loss_buf.p) ctx->loss_buf.alloc(sizeof(double));
            dl = ctx->loss_buf.as<double>();
        }
        float *dy = work, *dh = work + (size_t)batch * chess::kMlpOut;
        HIPCHECK(chess::launch_mlp_grad(params, x, hidden, y, target, batch, dy, dh, grad, dl, ctx->stream));
        if (loss) {
            HIPCHECK(hipMemcpyAsync(loss, dl, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
            HIPCHECK(hipStreamSynchronize(ctx->stream));
        }
    });
}

int chess_mlp_adam(chess_ctx *ctx, float *params, const float *grad, float *m, float *v, int64_t n,
                   float lr, float beta1, float beta2, float eps, int32_t step) {
    return chess::guarded(ctx, [&] {
        if (!params || !grad || !m || !v || n < 0 || step < 1)
            CHESS_THROW(CHESS_E_ARG, "mlp_adam: null pointer, negative size or step < 1");
        const double c1 = 1.0 - std::pow((double)beta1, step), c2 = 1.0 - std::pow((double)beta2, step);
        HIPCHECK(chess::launch_adam(params, grad, m, v, n, lr, beta1, beta2, eps, (float)c1, (float)c2, ctx->stream));
    });
}

int chess_model_load(chess_ctx *ctx, const float *blob, int64_t n) {
    return chess::guarded(ctx, [&] { chess::model_load(ctx, blob, n); });
}

int chess_model_save(const chess_ctx *ctx, float *blob, int64_t n) {
    if (!ctx || !blob || n != CHESS_MODEL_FLOATS) return CHESS_E_ARG;
    if (!ctx->model.loaded) return CHESS_E_ARG;
    std::memcpy(blob, ctx->model.blob.data(), sizeof(float) * CHESS_MODEL_FLOATS);
    return CHESS_OK;
}

}  // extern "C"
