/*
 * Oracle, matrix part: the Chebyshev matrix recursion on a fixed sparsity
 * pattern, in plain scalar CSR and float64.
 *
 * TEST INFRASTRUCTURE ONLY.  Called (through ctypes) by the tests, the smoke
 * check and the CPU-baseline leg of the benchmark; never by the product.  It
 * shares no code, header or table with the HIP path.
 *
 * What it computes, with the paper's definitions:
 *   - masked product (Sec. "Truncation to a fixed sparsity pattern"): after a
 *     product, every entry outside the target pattern is set to zero, i.e.
 *     C = P_C o (A B), computed only for (i, j) in P_C;
 *   - the recursion of Eq. 4 with that truncation, by left multiplication
 *     (columns obey the recursion independently, Sec. "Expansion in Chebyshev
 *     polynomials"):  T_0 = I, T_1 = M~ (placed in P_K),
 *     T_{k+1} = P_K o (2 M~ T_k) - T_{k-1};
 *   - the weighted sums of Eq. 1, acc_q = c_q[0]/2 T_0 + sum_{k>=1} c_q[k] T_k,
 *     for several coefficient sets at once (re-evaluation with new
 *     coefficients without new products, Sec. "Fermi Operator Expansion");
 *   - the moments t_k = Tr T_k (used for Tr W^p of Eq. 6 and for Tr(K) as a
 *     function of mu).
 *
 * Style: one row at a time, a dense marker array per thread (Gustavson's
 * row-by-row product), no blocking, no SIMD intrinsics.  OpenMP only splits
 * rows between threads; every sum runs in the same order as the serial loop.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* C = P_C o (A B) for square n x n CSR matrices.  Returns 0, or -1 if a
 * marker array cannot be allocated. */
int oracle_masked_spgemm(int64_t n,
                         const int64_t *arp, const int32_t *aci, const double *av,
                         const int64_t *brp, const int32_t *bci, const double *bv,
                         const int64_t *crp, const int32_t *cci, double *cv)
{
    int failed = 0;
#pragma omp parallel
    {
        int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        if (!mark) {
#pragma omp atomic write
            failed = 1;
        } else {
            for (int64_t j = 0; j < n; ++j) mark[j] = -1;
#pragma omp for schedule(dynamic, 64)
            for (int64_t i = 0; i < n; ++i) {
                for (int64_t p = crp[i]; p < crp[i + 1]; ++p) {
                    mark[cci[p]] = p;
                    cv[p] = 0.0;
                }
                for (int64_t q = arp[i]; q < arp[i + 1]; ++q) {
                    const int64_t l = aci[q];
                    const double a = av[q];
                    for (int64_t r = brp[l]; r < brp[l + 1]; ++r) {
                        const int64_t p = mark[bci[r]];
                        if (p >= 0) cv[p] += a * bv[r];
                    }
                }
                for (int64_t p = crp[i]; p < crp[i + 1]; ++p) mark[cci[p]] = -1;
            }
            free(mark);
        }
    }
    return failed ? -1 : 0;
}

/* Places a matrix given on pattern P_A into pattern P_B (P_A within P_B);
 * entries of P_B not in P_A become 0.  Returns -2 if P_A is not within P_B. */
int oracle_embed(int64_t n, const int64_t *arp, const int32_t *aci, const double *av,
                 const int64_t *brp, const int32_t *bci, double *bv)
{
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = brp[i]; p < brp[i + 1]; ++p) bv[p] = 0.0;
        int64_t p = brp[i];
        for (int64_t q = arp[i]; q < arp[i + 1]; ++q) {
            while (p < brp[i + 1] && bci[p] < aci[q]) ++p;
            if (p == brp[i + 1] || bci[p] != aci[q]) { bad = 1; break; }
            bv[p] = av[q];
        }
    }
    return bad ? -2 : 0;
}

static double trace_csr(int64_t n, const int64_t *rp, const int32_t *ci, const double *v)
{
    double t = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] == i) t += v[p];
    return t;
}

/*
 * The truncated Chebyshev chain of Eq. 4 and the sums of Eq. 1.
 *   mrp/mci/mv : M~ (already scaled and shifted, Eq. 2) on pattern P_M;
 *   krp/kci    : pattern P_K (must contain P_M and the diagonal);
 *   n_pl       : number of terms T_0 .. T_{n_pl-1};
 *   nq, coef   : nq coefficient sets, coef[q*n_pl + k];
 *   acc        : out, nq arrays of nnz(P_K) values (may be NULL if nq == 0);
 *   moments    : out, n_pl values t_k = Tr T_k (may be NULL);
 *   k_stop     : only T_0 .. T_{k_stop-1} are formed (k_stop = n_pl for the
 *                full chain; smaller values time a bounded sample).
 * Returns 0, -1 on allocation failure, -2 if P_M is not within P_K.
 */
int oracle_chebyshev(int64_t n,
                     const int64_t *mrp, const int32_t *mci, const double *mv,
                     const int64_t *krp, const int32_t *kci,
                     int32_t n_pl, int32_t nq, const double *coef,
                     double *acc, double *moments, int32_t k_stop)
{
    const int64_t nnz = krp[n];
    double *tm = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    double *t0 = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    double *t1 = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!tm || !t0 || !t1) { free(tm); free(t0); free(t1); return -1; }
    if (k_stop > n_pl) k_stop = n_pl;
    int rc = 0;

    /* T_0 = I on P_K */
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = krp[i]; p < krp[i + 1]; ++p) t0[p] = (kci[p] == i) ? 1.0 : 0.0;
    for (int32_t q = 0; q < nq; ++q)
        for (int64_t p = 0; p < nnz; ++p) acc[(size_t)q * nnz + p] = 0.5 * coef[(size_t)q * n_pl] * t0[p];
    if (moments) moments[0] = trace_csr(n, krp, kci, t0);

    if (k_stop > 1) {
        /* T_1 = M~ placed in P_K */
        rc = oracle_embed(n, mrp, mci, mv, krp, kci, t1);
        if (rc) goto done;
        for (int32_t q = 0; q < nq; ++q)
            for (int64_t p = 0; p < nnz; ++p) acc[(size_t)q * nnz + p] += coef[(size_t)q * n_pl + 1] * t1[p];
        if (moments) moments[1] = trace_csr(n, krp, kci, t1);
    }
    for (int32_t k = 1; k + 1 < k_stop; ++k) {
        /* tm = P_K o (M~ T_k) */
        rc = oracle_masked_spgemm(n, mrp, mci, mv, krp, kci, t1, krp, kci, tm);
        if (rc) goto done;
        /* T_{k+1} = 2 tm - T_{k-1}, stored over T_{k-1} */
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < nnz; ++p) t0[p] = 2.0 * tm[p] - t0[p];
        for (int32_t q = 0; q < nq; ++q) {
            const double c = coef[(size_t)q * n_pl + k + 1];
            double *a = acc + (size_t)q * nnz;
#pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < nnz; ++p) a[p] += c * t0[p];
        }
        if (moments) moments[k + 1] = trace_csr(n, krp, kci, t0);
        /* rotate: (T_{k-1}, T_k) <- (T_k, T_{k+1}) */
        double *sw = t0; t0 = t1; t1 = sw;
    }
done:
    free(tm); free(t0); free(t1);
    return rc;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the parallel regions above (for timing on fewer cores). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
