// Host-side scalar mathematics of the method: Chebyshev coefficients (Eq. 5)
// by a direct DCT, the degree rule (Eq. 7), occupation functions (Eqs. 9 and
// 11), the penalty function (Eq. 6), the electron count N(mu) from trace
// moments, the mu bisection and eigenvalue extraction, and the tridiagonal
// eigenproblem of the Lanczos bound estimate.  No device code here.
#pragma once
#include <cmath>
#include <functional>
#include <vector>

namespace chess {
namespace hostmath {

using Fn = std::function<double(double)>;

inline void scale_shift(double lo, double hi, double *sigma, double *tau) {
    *sigma = 2.0 / (hi - lo);
    *tau = 0.5 * (lo + hi);
}

// Eq. 5: c_j = 2/n sum_k f(cos(pi (k+1/2)/n)/sigma + tau) cos(pi j (k+1/2)/n),
// j = 0..n-1.  The cosines come from one table of cos(pi m / (2n)), m < 4n,
// indexed exactly by j (2k+1) mod 4n.
std::vector<double> cheb_coeffs(const Fn &f, double lo, double hi, int n);

// Same DCT applied to given samples fx[k] = f(x_k) at the Chebyshev nodes.
std::vector<double> cheb_coeffs_from_samples(const std::vector<double> &fx);

// Chebyshev nodes x_k of [lo, hi] (k = 0..n-1), in the order of Eq. 5.
std::vector<double> cheb_nodes(double lo, double hi, int n);

// sum' c_j T_j(x) by Clenshaw's recurrence (x already scaled to [-1, 1]).
double cheb_eval(const std::vector<double> &c, int m, double x);

// Number of Chebyshev-Lobatto points on which Eq. 7's maximum is taken for
// an m-term fit: max(8192, 8 m).  The error curve of an m-term interpolant
// has about m oscillations over [lo, hi], so the grid samples each of them
// about 8 times (a fixed grid would miss the peaks once m nears its size).
inline int fit_points(int m) { return m > 1024 ? 8 * m : 8192; }

// max |p_m - f| over npts Chebyshev-Lobatto points of [lo, hi] (npts <= 0:
// fit_points(m)).
double fit_error(const Fn &f, double lo, double hi, int m, int npts = 0);

// Eq. 7: smallest m (a multiple of `step`) with fit_error < tol; doubling then
// bisection over multiples of `step` (the error decreases with m for the
// functions used here).  Returns -1 if m_max does not reach tol.
int degree(const Fn &f, double lo, double hi, double tol, int step, int m_max, int npts = 0);

// Occupations, Eqs. 11 and 9 (reading: beta = 1/kT).
inline double occ_erfc(double e, double mu, double kT) { return 0.5 * std::erfc((e - mu) / kT); }
inline double occ_fd(double e, double mu, double kT) {
    const double x = (e - mu) / kT;
    if (x > 0) {
        const double ex = std::exp(-x);
        return ex / (1.0 + ex);
    }
    return 1.0 / (1.0 + std::exp(x));
}

// Electron count from trace moments: N(mu) = sum' c_j(mu) t_j.  Writing c_j
// out as the DCT of Eq. 5 gives N(mu) = 2/n sum_m f(x_m; mu) g_m with
// g_m = t_0/2 + sum_{j>=1} t_j cos(j theta_m), which does not depend on mu:
// one DCT up front, then O(n) (or less) per evaluation.
struct CountFunction {
    double lo = 0, hi = 0, kT = 0;
    int smearing = 0;  // 0 erfc, 1 Fermi-Dirac
    std::vector<double> x;   // nodes, descending
    std::vector<double> g;   // weights g_m
    std::vector<double> cum; // cum[m] = sum_{m' < m} g_m'  (nodes above x_m)
    void init(const std::vector<double> &moments, double lo, double hi, double kT, int smearing);
    // exact sum over all nodes
    double operator()(double mu) const;
    // nodes farther than `cut` kT from mu are taken as fully occupied/empty
    double local(double mu) const;
};

// Bisection for N(mu) = target on [a, b]; returns false if not bracketed.
bool bisect_mu(const CountFunction &N, double target, double tol_n, double a, double b,
               double *mu, int *iters);

// Eigenvalues: for each integer N with N(e_lo) < N - 1/2 < N(e_hi), the mu
// solving N(mu) = N - 1/2 (Sec. "Extraction of selected eigenvalues").
std::vector<double> eigenvalues(const CountFunction &N, double e_lo, double e_hi, double tol_e);

// Penalty trace of Eq. 6 in the scaled variable (bounds -1 and 1):
// Tr W^p = sum' c^p_j t_j with f^p(x) = exp(alpha (x + 1)) - exp(-alpha (x - 1)).
// Also returns the fit error of f^p with min(n, 1024) terms (beyond about
// 1024 terms the fit of this entire function is at rounding level).
double penalty_trace(const std::vector<double> &moments, double alpha, double *fit_err);

// The check of the spectral bounds on the moments t_k = Tr T_k of one chain
// over n_rows rows (Sec. "Determination of the eigenvalue bounds and
// polynomial degree", Eq. 6, alpha = -200 in the scaled variable, where an
// eigenvalue at a bound contributes 1):
//   growth test first: |T_k| <= 1 on [-1, 1], so |Tr T_k| > 1.01 n_rows for
//     some k means an eigenvalue outside the bounds.  Then the penalty's value
//     is decided by rounding noise in its coefficients times that growth, so
//     the side comes from the moments themselves: T_k(x) alternates in sign
//     for x < -1 and keeps one sign for x > 1 (last 16 moments);
//   otherwise, when the fit of f^p is good enough (valid: n_rows * fit error
//     < 0.1), |Tr W^p| > 0.5 fails the check and its sign picks the side
//     (positive: an eigenvalue at or below the lower bound).
//   side: -1 move the lower bound, +1 the upper one, when not ok.
struct BoundsCheck {
    bool ok = true, valid = false;
    double penalty = NAN;
    int side = 0;
};
BoundsCheck bounds_check(const std::vector<double> &moments, long long n_rows);

// Terms with which Eq. 6 is trusted on n_rows rows: the fewest multiple of 8
// (at most 1024) whose fit of f^p (alpha = -200, bounds -1 and 1) has
// n_rows * fit error < 0.1.  A matrix-power series shorter than this is
// judged on a moments-only chain of this many terms before it is summed.
int penalty_degree(long long n_rows);

// Moves the failing side out by 10 % of the width (side 0: both).
inline void widen(int side, double *lo, double *hi) {
    const double w = *hi - *lo;
    if (side <= 0) *lo -= 0.1 * w;
    if (side >= 0) *hi += 0.1 * w;
}

// Extreme eigenvalues of the symmetric tridiagonal matrix (alpha, beta) by
// Sturm bisection, and the residual |beta_last * s_last| of their Ritz vectors.
void tridiag_extremes(const std::vector<double> &alpha, const std::vector<double> &beta,
                      double beta_last, double *tmin, double *tmax, double *rmin, double *rmax);

}  // namespace hostmath
}  // namespace chess
