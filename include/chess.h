/*
 * chess.h -- C interface of the Chebyshev sparse matrix-function library for
 * AMD Instinct MI355X (gfx950).
 *
 * The library evaluates f(M) for a sparse symmetric matrix M by the Chebyshev
 * expansion of the paper "Efficient computation of sparse matrix functions for
 * large scale electronic structure calculations: The CheSS library":
 *
 *   p(M) = c_0/2 I + sum_{j=1}^{n_pl-1} c_j T_j(M~)          (Eq. 1)
 *   M~ = sigma (M - tau I), sigma = 2/(e_max-e_min),
 *   tau = (e_min+e_max)/2                                     (Eqs. 2-3)
 *   T_0 = I, T_1 = M~, T_{j+1} = 2 M~ T_j - T_{j-1}            (Eq. 4)
 *   c_j from f at the Chebyshev nodes                         (Eq. 5)
 *
 * Every product is truncated to a fixed block sparsity pattern (Sec.
 * "Truncation to a fixed sparsity pattern"), so T_j and p(M) live on the
 * caller's output pattern.
 *
 * Conventions for every entry point
 * ---------------------------------
 * Matrices are block CSR with a uniform block edge b (4 or 9: one block per
 * atom pair).  A pattern is square, its column indices are strictly increasing
 * in each block row, every diagonal block is present and the pattern is
 * structurally symmetric.  Values are nnzb*b*b numbers, blocks in pattern
 * order, each block row-major.  All pointers inside chess_pattern and
 * chess_matrix are DEVICE pointers on the context's device; pointers marked
 * "host" below are host memory.  The caller allocates and frees every input
 * and output; the library never frees or keeps caller memory beyond a call.
 * Workspace (and cached per-pattern plans) belongs to the context.
 *
 * Work is ordered on the context's stream.  Every entry point returns after
 * the stream has drained (results that reach the host, such as mu or
 * eigenvalues, need that anyway), so outputs are ready on return.  A context
 * must not be used by two threads at once; different contexts (on one device
 * or several) may be used from different threads at the same time.
 *
 * Errors: every call returns CHESS_OK (0) or a negative CHESS_E_* code; then
 * chess_last_error() describes it and the outputs are undefined.
 */
#ifndef CHESS_H
#define CHESS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CHESS_OK = 0,
    CHESS_E_ARG = -1,         /* bad argument: null pointer, size mismatch, b mismatch */
    CHESS_E_PATTERN = -2,     /* unsorted/asymmetric pattern, missing diagonal, pattern not nested */
    CHESS_E_NOT_SPD = -3,     /* a non-integer power of a matrix whose lower bound is not > 0 */
    CHESS_E_BOUNDS = -4,      /* spectral bounds still fail after max_reexpand widenings */
    CHESS_E_NOCONV = -5,      /* mu search did not bracket or converge */
    CHESS_E_OOM = -6,         /* device allocation failed */
    CHESS_E_HIP = -7,         /* a HIP runtime call failed */
    CHESS_E_UNSUPPORTED = -8, /* block edge not 4 or 9, dtype not CHESS_F64, row too long */
    CHESS_E_CAPACITY = -9     /* eigenvalue buffer too small; *n_found holds the count */
};

/* Precision of the Chebyshev chain.  Inputs and outputs are always float64,
 * and so are the weighted sums of Eq. 1, the traces and the bound/mu logic.
 *   CHESS_F64    : float64 chain;
 *   CHESS_F32    : T_k stored and multiplied in float32;
 *   CHESS_BF16   : T_k stored in float32, each product's operands rounded to
 *                  bfloat16 (nearest even), float32 accumulation on the
 *                  matrix cores (block edge 4 only);
 *   CHESS_BF16X3 : T_k in float32, each operand x split as hi = bf16(x),
 *                  lo = bf16(x - hi) and the product taken as
 *                  hi*hi + hi*lo + lo*hi, float32 accumulation (block edge
 *                  4 only).
 * Default Eq. 7 thresholds: 1e-10 (F64), 1e-6 (F32, BF16X3), 1e-4 (BF16).
 * The bfloat16 forms return CHESS_E_UNSUPPORTED for b = 9 or rows of more
 * than 254 blocks. */
enum { CHESS_F64 = 0, CHESS_F32 = 1, CHESS_BF16 = 2, CHESS_BF16X3 = 3 };

/* Occupation function for the Fermi-operator expansion. */
enum {
    CHESS_ERFC = 0,        /* Eq. 11: f = 1/2 erfc((e - mu)/kT) */
    CHESS_FERMI_DIRAC = 1  /* Eq. 9:  f = 1/(1 + exp((e - mu)/kT)) */
};

/* How bounds that are not given are estimated (Sec. "Determination of the
 * eigenvalue bounds and polynomial degree"). */
enum {
    CHESS_BOUNDS_GERSHGORIN = 0, /* Gershgorin discs: rigorous, wide */
    CHESS_BOUNDS_LANCZOS = 1,    /* a few Lanczos steps plus a margin: tight, checked by Eq. 6 */
    CHESS_BOUNDS_LEARNED = 2,    /* the loaded predictor (chess_model_load): bounds and a mu
                                    bracket from matrix statistics, checked by Eq. 6 and the
                                    growth test; the Gershgorin interval is the fallback */
    CHESS_BOUNDS_LEARNED_LANCZOS = 3 /* the predictor's interval intersected with the
                                    CHESS_BOUNDS_LANCZOS one, and its mu bracket; when Eq. 6 or
                                    the growth test rejects the intersection, the Lanczos
                                    interval (batched calls: the Gershgorin one) */
};

typedef struct chess_ctx chess_ctx;

typedef struct {
    int32_t b;              /* block edge: 4 or 9 */
    int32_t nbrows;         /* number of block rows (= block columns) */
    int64_t nnzb;           /* number of stored blocks */
    const int64_t *row_ptr; /* device, nbrows+1 entries, row_ptr[0] = 0 */
    const int32_t *col_idx; /* device, nnzb entries */
} chess_pattern;

typedef struct {
    chess_pattern pat;
    void *val;     /* device, nnzb*b*b values (const for inputs) */
    int32_t dtype; /* must be CHESS_F64 */
} chess_matrix;

typedef struct {
    int32_t precision;   /* CHESS_F64, CHESS_F32 (default), CHESS_BF16 or CHESS_BF16X3 */
    int32_t smearing;    /* CHESS_ERFC (default) or CHESS_FERMI_DIRAC */
    int32_t bounds_mode; /* for bounds not given (default CHESS_BOUNDS_GERSHGORIN) */
    int32_t n_pl;        /* > 0: fixed number of terms for H (or M); 0: Eq. 7 */
    int32_t n_pl_s;      /* > 0: fixed number of terms for the S^-1/2 chain; 0: Eq. 7 */
    int32_t store_history;   /* 1: keep every T_k (float32/float64) and recombine after the
                                mu search (one chain pass); 0: second pass at the final mu */
    int32_t max_reexpand;    /* widenings allowed when Eq. 6 or the growth test fails (3) */
    int32_t lanczos_steps;   /* Lanczos steps for CHESS_BOUNDS_LANCZOS and for S (40) */
    double tol_fit;      /* Eq. 7 threshold for H (<= 0: by precision, see above) */
    double tol_fit_s;    /* Eq. 7 threshold for x^-1/2 or x^a (<= 0: same rule) */
    double tol_ne;       /* |N(mu) - N_e| target of the mu search (<= 0: 1e-8 N_e) */
    double bounds[2];    /* spectral bounds of H' = S^-1/2 H S^-1/2 (or of M); NaN = estimate */
    double s_bounds[2];  /* spectral bounds of S; NaN = estimate */
    double mu;           /* not NaN: use this mu, no search */
    double mu_bracket[2];/* not NaN: search mu here first, fall back to the full bounds */
    double eig_width;    /* kT of the occupation used to extract eigenvalues (1e-3) */
    double bound_margin; /* relative margin added to Lanczos bounds (0.02) */
    /* Width check of Sec. "Fermi Operator Expansion" (chess_fermi_operator):
     * after mu is found for kT, E = Tr(K' H') is compared with E' for the
     * wider occupation kt_ratio * kT (its own mu for the same N); both come
     * from the moments of the same chain, which runs one term longer.  While
     * |E - E'| > tol_energy, kT is halved and the expansion redone (a new
     * degree unless n_pl is given), at most max_kt_halvings times. */
    int32_t adapt_kt;        /* 1: check and adapt the width (default 0) */
    int32_t max_kt_halvings; /* (4) */
    double kt_ratio;         /* kT'/kT of the second occupation (> 1; default 1.25) */
    double tol_energy;       /* |E - E'| threshold in Ha (<= 0: 1e-4 N_e) */
    /* Warm start (chess_fermi_operator, chess_eigs_in_interval): in an SCF
     * cycle S does not change, so S^-1/2 from an earlier call can be given
     * back and the S chain is skipped (Sec. "Determination of the eigenvalue
     * bounds and polynomial degree": guesses from the previous iteration;
     * the bounds and a mu bracket go in bounds / mu_bracket).  Both are
     * device arrays of float64 on `pattern` (nnzb * b * b values, blocks in
     * pattern order, row-major), owned by the caller; NULL = not used.
     * With CHESS_BOUNDS_LEARNED and sinvhalf_in, s_bounds must be given. */
    const void *sinvhalf_in; /* S^-1/2 to use instead of computing it */
    void *sinvhalf_out;      /* receives the S^-1/2 the call used */
} chess_opts;

typedef struct {
    double mu;            /* chemical potential used */
    double lo, hi;        /* bounds used for H' (or M) */
    double s_lo, s_hi;    /* bounds used for S */
    double tr_ks;         /* Tr(K S) of the returned K */
    double ne_chain;      /* N(mu) from the moments of the chain */
    double penalty;       /* Tr W^p of Eq. 6 for the final bounds (NaN if not evaluated) */
    int32_t n_pl, n_pl_s; /* terms used */
    int32_t passes;       /* chain passes over H~' */
    int32_t bisect_iters; /* mu search iterations */
    int32_t reexpansions; /* bound widenings */
    int32_t chain_steps;  /* products launched in chains (all matrices) */
    double ms_total, ms_setup, ms_s_chain, ms_transform, ms_h_chain, ms_mu, ms_post;
    double ms_chain_kernel; /* summed device time of the H~' chain product kernel */
    int32_t kernel_variant; /* variant of the chain product kernel chosen by timing, or
                               forced by CHESS_LISTED_VARIANT in the environment
                               (-1: the searching kernel) */
    int32_t fallback;       /* CHESS_BOUNDS_LEARNED: bit 0 = predicted bounds rejected (Eq. 6
                               or growth test) and replaced by the Gershgorin interval,
                               bit 1 = mu not inside the predicted bracket */
    double pred_lo, pred_hi, pred_mu; /* predictor outputs (NaN unless CHESS_BOUNDS_LEARNED) */
    double ms_learned;      /* features + inference time */
    double energy;          /* adapt_kt: E = Tr(K' H') at the returned kT (NaN otherwise) */
    double energy_wide;     /* adapt_kt: E' at kt_ratio times the returned kT */
    double kt_used;         /* kT of the returned K */
    int32_t kt_halvings;    /* adapt_kt: halvings of kT taken */
    /* chess_fermi_operator and, per system, chess_fermi_operator_batched:
     * rough HOMO and LUMO in Ha from the same moments
     * (Sec. "Extraction of selected eigenvalues": the polynomials already
     * computed give such estimates almost for free).  With N_h = ceil(N_e)
     * states occupied, homo solves N(e) = N_h - 1/2 and lumo N(e) = N_h + 1/2
     * with the call's occupation function at the returned kT.  They are
     * accurate only for states isolated by several kT from their neighbours;
     * NaN if N_h is 0 (homo) or n (lumo), and in the other entry points.
     * In a batch they come from the system's first attempt, or from the
     * Gershgorin redo when its bounds were rejected. */
    double homo, lumo;
    /* chess_fermi_operator: the part of ms_chain_kernel spent in passes that
     * accumulate K' (the moments-only passes make up the rest); 0 elsewhere */
    double ms_chain_kernel_acc;
    /* chess_fermi_operator: chain kernel variant of the moments-only passes
     * (kernel_variant is that of the last pass; -1 if there was none) */
    int32_t kernel_variant_moments;
    /* chess_fermi_operator: rows per tile of the H~' chain's plan (b = 4: 4 or
     * 2, chosen by timing on the first chain over a pattern, or forced by
     * CHESS_TILE_ROWS = 1, 2 or 4 in the environment; 0 for the searching
     * kernel) */
    int32_t tile_rows;
    /* chess_fermi_operator: product launches of the moments-only passes; such
     * a pass runs half its chain (n_pl / 2 - 1 products) and takes the other
     * moments from Frobenius products of the T_m it computed */
    int32_t moment_products;
    /* chess_matrix_power, and the S chain of chess_fermi_operator,
     * chess_eigs_in_interval and each item of chess_fermi_operator_batched:
     * Tr W^p of Eq. 6 for the final bounds of S (NaN if not evaluated, e.g.
     * with sinvhalf_in) and the number of moments it was judged on: the
     * series' own n_pl_s terms, or, when that is fewer than Eq. 6 needs on
     * this many rows (chess_degree with CHESS_FN_PENALTY), a moments-only
     * chain of that many terms run first (in batches always the latter) */
    double s_penalty;
    int32_t s_check_terms;
} chess_info;

/*
 * A batch of independent systems (each as in chess_fermi_operator) that
 * share the work of one call: per block edge b, the systems are laid out
 * block-diagonally and every chain runs once over the whole batch - one S
 * chain giving S^-1/2 and S^-1 (Sec. "Matrix powers": both powers from the
 * same T_k), one chain on H~' accumulating K' at three trial chemical
 * potentials (Eq. 1 with three coefficient sets on the same T_k), with the
 * moments Tr T_k of every system, and the sandwich products of Sec. "Fermi
 * Operator Expansion" run once over the batch.  Row tiles never straddle
 * systems, so each system keeps its own bounds, degree n_pl (terms past it
 * have zero weight), coefficients and moments.  The products of each chain
 * after the first are recorded into one HIP graph and launched as one graph
 * (CHESS_BATCH_GRAPH=0 in the environment launches them one by one).  The
 * kernel variant is chosen by timing as for single systems.
 * Per system (all matrices device, float64):
 *   H, S, pattern, n_electrons, kT : as for chess_fermi_operator
 *   mu_trial[3] : chemical potentials at which K is formed; NaN entries take
 *                 mu^ - d, mu^, mu^ + d from the loaded predictor
 *                 (opts->bounds_mode = CHESS_BOUNDS_LEARNED, d = its bracket
 *                 half width), otherwise CHESS_E_ARG
 *   K_out[3]    : K at mu_trial[q] on exactly `pattern`, or NULL (not formed)
 *   Sinvhalf_out, Sinv_out : S^-1/2 and S^-1 on `pattern`, or NULL
 *   ne_trial    : host, 3 doubles or NULL: N(mu_trial[q]) from the moments
 *   info        : host or NULL: mu = the root of N(mu) = N_e from the moments,
 *                 lo, hi, s_lo, s_hi, n_pl, n_pl_s, penalty, tr_ks (of K at
 *                 mu_trial[1]), ne_chain = N(mu_trial[1]), s_penalty,
 *                 s_check_terms, reexpansions (of S); ms_total and
 *                 ms_chain_kernel are those of the whole call
 * The bounds of each S are judged as in chess_matrix_power, on one
 * moments-only check chain over the batch (each system to the terms Eq. 6
 * needs on its rows); failing systems widen and the check runs again, at
 * most max_reexpand times, else CHESS_E_BOUNDS.
 * A system whose bounds of H' fail Eq. 6 or the growth test is redone, after
 * the others, in a batch of its own with the Gershgorin interval
 * (info->fallback bit 0 set); CHESS_E_BOUNDS only if the Gershgorin interval
 * itself fails.  opts apply to every system.
 */
typedef struct {
    const chess_matrix *H;
    const chess_matrix *S;
    const chess_pattern *pattern;
    double n_electrons;
    double kT;
    double mu_trial[3];
    chess_matrix *K_out[3];
    chess_matrix *Sinvhalf_out;
    chess_matrix *Sinv_out;
    double *ne_trial;
    chess_info *info;
} chess_batch_item;

int chess_fermi_operator_batched(chess_ctx *ctx, int32_t nsys, const chess_batch_item *items,
                                 const chess_opts *opts);

/*
 * Learned predictor of the spectral bounds and of mu.
 *
 * The paper notes that good initial bounds avoid recomputing the expansion
 * after a failed Eq. 6 check (Sec. "Determination of the eigenvalue bounds and
 * polynomial degree") and save the bound search (Sec. "Scaling with spectral
 * properties").  A two-layer perceptron maps CHESS_N_FEATURES statistics of H'
 * (Gershgorin interval, diagonal and radius histograms, Tr T_k for k <= 8,
 * kT, filling, size) to (eps_min, eps_max, mu) in units of the Gershgorin
 * interval: y = c + w * (W2 tanh(W1 x~ + b1) + b2) * y_std + y_mean, with
 * x~ = (x - x_mean) * x_inv_std, c and w the centre and half width.
 *
 * Parameter vector (float32, CHESS_MLP_PARAMS): W1 [128][64], b1 [128],
 * W2 [3][128], b2 [3], row-major.  Normalisation block (CHESS_MLP_NORM):
 * x_mean [64], x_inv_std [64], y_mean [3], y_std [3].
 * Model blob (CHESS_MODEL_FLOATS): normalisation block, then
 * {margin_lo, margin_hi, mu_half} in Gershgorin half widths, then the
 * parameters.  Bounds used: [eps_min - margin_lo w, eps_max + margin_hi w]
 * clipped to the Gershgorin interval; mu bracket: mu -+ mu_half w.
 */
#define CHESS_N_FEATURES 64
#define CHESS_MLP_HIDDEN 128
#define CHESS_MLP_OUT 3
#define CHESS_MLP_PARAMS (128 * 64 + 128 + 3 * 128 + 3)
#define CHESS_MLP_NORM (2 * 64 + 2 * 3)
#define CHESS_MODEL_FLOATS (CHESS_MLP_NORM + 3 + CHESS_MLP_PARAMS)

/*
 * Features of (H, S) on `pattern` (as for chess_fermi_operator): builds the
 * orthogonal frame (S^-1/2 chain, H'), then the statistics listed above.
 *   feat_out  : host, CHESS_N_FEATURES floats
 *   gersh_out : host, 2 doubles (Gershgorin interval of H'), may be NULL
 * Synchronises before returning.
 */
int chess_features(chess_ctx *ctx, const chess_matrix *H, const chess_matrix *S,
                   const chess_pattern *pattern, double n_electrons, double kT, float *feat_out,
                   double *gersh_out, const chess_opts *opts);

/*
 * Perceptron forward pass on `batch` rows (all pointers device, float32):
 *   x [batch][64] -> y [batch][3]; hidden [batch][128] receives the tanh
 *   outputs if not NULL; norm (CHESS_MLP_NORM floats) applies the
 *   normalisation block, NULL = identity.  Stream-ordered (no wait).
 */
int chess_mlp_forward(chess_ctx *ctx, const float *params, const float *norm, const float *x,
                      int32_t batch, float *hidden, float *y);
/*
 * Gradient of L = 1/(2 batch) sum (y - target)^2 with respect to the
 * parameters, from a forward pass without normalisation (x, hidden, y as it
 * wrote them).  work: device, batch * (3 + 128) floats of scratch owned by
 * the caller; grad: device, CHESS_MLP_PARAMS floats (overwritten); loss: host,
 * may be NULL (when given, the call waits for it).  Sums over the batch run
 * in a fixed order in float64.
 */
int chess_mlp_grad(chess_ctx *ctx, const float *params, const float *x, const float *hidden,
                   const float *y, const float *target, int32_t batch, float *work, float *grad,
                   double *loss);
/*
 * Adam step `step` (1, 2, ...) on n parameters (device): m, v are the moment
 * estimates (zero before step 1), bias-corrected.  Stream-ordered.
 */
int chess_mlp_adam(chess_ctx *ctx, float *params, const float *grad, float *m, float *v, int64_t n,
                   float lr, float beta1, float beta2, float eps, int32_t step);
/*
 * chess_mlp_grad without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving or training
 * loops, harnesses that forbid hipMalloc): the same kernels and result as
 * chess_mlp_grad, with the workspace (and the loss on the device) taken from
 * a fixed array inside the library instead of `work` and the context.
 * batch must be 1..CHESS_NOALLOC_MAX_BATCH (else CHESS_E_ARG); the array
 * holds 256 + CHESS_NOALLOC_MAX_BATCH * 131 * 4 bytes per GPU for the life of
 * the process.  Every call on one GPU shares that array: calls that overlap
 * on one GPU (from several contexts or threads) race.  loss (host, may be
 * NULL): when given, the call waits for it; with NULL it only enqueues
 * kernels on the context's stream.
 */
#define CHESS_NOALLOC_MAX_BATCH 4096
int chess_mlp_grad_noalloc(chess_ctx *ctx, const float *params, const float *x, const float *hidden,
                           const float *y, const float *target, int32_t batch, float *grad,
                           double *loss);
/* Loads a model blob (host, n = CHESS_MODEL_FLOATS) into the context for
 * CHESS_BOUNDS_LEARNED; CHESS_E_ARG for a wrong size, non-finite entries or a
 * non-positive inverse scale.  chess_model_save copies the loaded blob back. */
int chess_model_load(chess_ctx *ctx, const float *blob, int64_t n);
int chess_model_save(const chess_ctx *ctx, float *blob, int64_t n);

/*
 * Degree rule of Eq. 7 (Sec. "Determination of the eigenvalue bounds and
 * polynomial degree"), host only, no context, no device work: the smallest
 * n_pl, a multiple of 8 up to 20000, whose Eq. 5 interpolant p of f on
 * [lo, hi] has max |p - f| < tol_fit over max(8192, 8 n_pl) Chebyshev-Lobatto
 * points of [lo, hi].  The entry points above use this rule wherever n_pl or
 * n_pl_s is not given.
 *   fn     : CHESS_FN_ERFC or CHESS_FN_FERMI_DIRAC: the occupation (Eq. 11 or
 *            Eq. 9) of width kT = param centred at mu = (lo + hi)/2, where the
 *            Chebyshev nodes are sparsest (the degree used for any mu);
 *            CHESS_FN_POWER: x^param (Sec. "Matrix powers"), lo > 0 needed
 *            unless param is a non-negative integer;
 *            CHESS_FN_PENALTY: the terms with which Eq. 6 is trusted on
 *            param rows: the smallest multiple of 8 (at most 1024) for which
 *            param times the fit error of the penalty function (alpha = -200,
 *            bounds -1 and 1, same grid rule) is below 0.1 (lo, hi and
 *            tol_fit must still be valid but are not used)
 *   n_pl_out : host, receives the degree
 * Returns CHESS_E_ARG for an unknown fn, hi <= lo, tol_fit <= 0, param <= 0
 * for an occupation, lo <= 0 for a non-integer power, param < 1 for
 * CHESS_FN_PENALTY, or a null n_pl_out; CHESS_E_NOCONV when 20000 terms do
 * not reach tol_fit.
 */
enum { CHESS_FN_ERFC = 0, CHESS_FN_FERMI_DIRAC = 1, CHESS_FN_POWER = 2, CHESS_FN_PENALTY = 3 };
int chess_degree(int32_t fn, double param, double lo, double hi, double tol_fit, int32_t *n_pl_out);

/* Fills *opts with the defaults listed above. */
void chess_default_opts(chess_opts *opts);

/* Creates a context on `device` that orders its work on `hip_stream`
 * (a hipStream_t; NULL = the null stream). */
int chess_create(chess_ctx **ctx, int device, void *hip_stream);
int chess_destroy(chess_ctx *ctx);
/*
 * Progress report from inside a chain: after every `every` products of a
 * chain the library waits for the stream and calls fn(user, stage, done,
 * total), with stage a static string naming the chain ("S chain", "H chain",
 * "H chain (accumulate)", ...), done the number of terms formed and total
 * the chain length n_pl. fn runs on the calling thread and must not call
 * back into the library. fn = NULL switches reporting off. Returns
 * CHESS_E_ARG for a NULL ctx or for every <= 0 with a non-NULL fn. The extra
 * waits cost one stream synchronisation per `every` products.
 */
typedef void (*chess_progress_fn)(void *user, const char *stage, int64_t done, int64_t total);
int chess_set_progress(chess_ctx *ctx, chess_progress_fn fn, void *user, int32_t every);

/* Message for the last non-zero return on this context (never NULL). */
const char *chess_last_error(const chess_ctx *ctx);

/*
 * Density kernel by Fermi-operator expansion (Sec. "Fermi Operator
 * Expansion"): K = S^-1/2 f(H~') S^-1/2 with H' = S^-1/2 H S^-1/2, f the
 * occupation (Eq. 11 or Eq. 9) and mu chosen so that Tr K' = N_e, where
 * K' = f(H~') (equal to Tr(KS) up to truncation).
 *   H, S    : on the same or different patterns, each contained in `pattern`;
 *   pattern : the kernel pattern P_K (also that of S^-1/2 and of every T_k);
 *   K_out   : caller-allocated on exactly `pattern` (same nbrows/nnzb/b).
 * opts may be NULL (defaults); info may be NULL.
 */
int chess_fermi_operator(chess_ctx *ctx, const chess_matrix *H, const chess_matrix *S,
                         const chess_pattern *pattern, double n_electrons, double kT,
                         chess_matrix *K_out, chess_info *info, const chess_opts *opts);

/*
 * Matrix power S^a for any real a (Sec. "Matrix powers"): the same expansion
 * with f(x) = x^a over the spectral bounds of S; non-integer or negative a
 * need a positive lower bound (else CHESS_E_NOT_SPD).  Sa_out is on `pattern`.
 * The bounds, degree and Eq. 7 threshold are those of S in opts: s_bounds,
 * n_pl_s, tol_fit_s.  The bounds are judged by the growth test and Eq. 6
 * (Sec. "Determination of the eigenvalue bounds and polynomial degree") on at
 * least the moments Eq. 6 needs on this many rows: a shorter series is first
 * checked on a moments-only chain of that length.  Bounds that fail move out:
 * both sides by 10 % of the width after the growth test, the penalty's side
 * by 2.5 % after Eq. 6, the lower bound at most halved; up to max_reexpand
 * times, else CHESS_E_BOUNDS.  info: lo, hi, n_pl, reexpansions, penalty
 * (= s_penalty), s_check_terms, chain_steps (check chains included).
 */
int chess_matrix_power(chess_ctx *ctx, const chess_matrix *S, double a,
                       const chess_pattern *pattern, chess_matrix *Sa_out,
                       chess_info *info, const chess_opts *opts);

/*
 * Eigenvalues of H c = e S c inside [lo, hi] (Sec. "Extraction of selected
 * eigenvalues"): the chain's trace moments give N(mu) = Tr f(H~'; mu) for any
 * mu; eigenvalue number N is the mu with N(mu) = N - 1/2.  `pattern` is the
 * pattern of S^-1/2 and of the T_k.  eig_out (host) receives the values in
 * ascending order; if more than `capacity` lie in the interval the call
 * returns CHESS_E_CAPACITY with *n_found set to the count.
 */
int chess_eigs_in_interval(chess_ctx *ctx, const chess_matrix *H, const chess_matrix *S,
                           double lo, double hi, const chess_pattern *pattern,
                           double *eig_out, int64_t capacity, int64_t *n_found,
                           chess_info *info, const chess_opts *opts);

/*
 * The Chebyshev chain itself (Eqs. 1, 4), for a matrix already in [-1, 1]:
 * M~ = sigma (M - tau I) with sigma, tau from the given bounds [lo, hi].
 *   M       : input on a pattern contained in `pattern`;
 *   n_pl    : terms T_0 .. T_{n_pl-1};
 *   coef    : host, nq sets of n_pl coefficients, coef[q*n_pl + k] (nq <= 4);
 *   acc_out : nq matrices on `pattern` receiving c_q[0]/2 I + sum c_q[k] T_k
 *             (may be NULL when nq == 0);
 *   moments : host, n_pl values Tr T_k (may be NULL).
 * The products run in opts->precision.
 */
int chess_chebyshev(chess_ctx *ctx, const chess_matrix *M, double lo, double hi,
                    const chess_pattern *pattern, int32_t n_pl, int32_t nq,
                    const double *coef, chess_matrix *acc_out, double *moments,
                    const chess_opts *opts);

/*
 * The truncated product (Sec. "Truncation to a fixed sparsity pattern"):
 * C = P_C o (A B), computed only on C's pattern, float64.  A, B, C must have
 * the same b and nbrows.
 */
int chess_masked_product(chess_ctx *ctx, const chess_matrix *A, const chess_matrix *B,
                         chess_matrix *C);

/*
 * Segment Storage Format (Sec. "Storage format of the sparse matrices"), for
 * callers that hold matrices the way CheSS stores them.  Host arrays only, no
 * context, no device work.  SSF: nseg segments of consecutive non-zero
 * entries of an n x n matrix, keyg [nseg][4] = (c_s, c_e, r_s, r_e), 1-based,
 * a segment running in row-major order from (r_s, c_s) to (r_e, c_e) (it may
 * continue over a row end); segments sorted and not overlapping; values in
 * one array of nval entries; keyv [nseg] (1-based) where each segment starts
 * in it, or NULL for one after the other.
 *
 * chess_ssf_to_bcsr: block CSR of edge b (n a multiple of b): block (I, J)
 * is stored when any entry inside it is; the others of a stored block are 0.
 *   row_ptr [n/b + 1], col_idx [capacity], val_bcsr [capacity * b * b]
 *   (row-major blocks in pattern order); all three NULL: only *nnzb_out is
 *   set.  CHESS_E_CAPACITY when capacity < nnzb (then *nnzb_out holds it);
 *   CHESS_E_ARG for segments out of range, unsorted, overlapping or reaching
 *   past nval.
 * chess_bcsr_to_ssf: one segment per maximal run of consecutive block columns
 *   in every scalar row (nseg = b * runs), keyv filled, values in segment
 *   order.  keyg [capacity][4], keyv [capacity], val [*nval_out]; all three
 *   NULL: only *nseg_out and *nval_out are set.  CHESS_E_CAPACITY when
 *   capacity < nseg; CHESS_E_ARG for a malformed pattern (row_ptr not
 *   starting at 0 or decreasing, columns out of range or not increasing).
 */
int chess_ssf_to_bcsr(int32_t b, int64_t n, int64_t nseg, const int64_t *keyg, const int64_t *keyv,
                      const double *val, int64_t nval, int64_t *row_ptr, int32_t *col_idx,
                      double *val_bcsr, int64_t capacity, int64_t *nnzb_out);
int chess_bcsr_to_ssf(int32_t b, int32_t nbrows, const int64_t *row_ptr, const int32_t *col_idx,
                      const double *val_bcsr, int64_t *keyg, int64_t *keyv, double *val, int64_t capacity,
                      int64_t *nseg_out, int64_t *nval_out);

#ifdef __cplusplus
}
#endif
#endif /* CHESS_H */
