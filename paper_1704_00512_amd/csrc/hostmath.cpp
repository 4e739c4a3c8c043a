// Host-side scalar mathematics (see hostmath.h).
#include "hostmath.h"

#include <algorithm>
#include <cmath>
#include <thread>

namespace chess {
namespace hostmath {

namespace {
constexpr double kPi = 3.14159265358979323846;

// fn(i) for i in [0, n): large loops are split over up to 16 host threads,
// each index written by exactly one thread (results do not depend on the
// split).
template <typename F>
void parallel_for(int n, F &&fn) {
    const int nt = (n >= 512) ? (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency())) : 1;
    if (nt <= 1) {
        for (int i = 0; i < n; ++i) fn(i);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            for (int i = t; i < n; i += nt) fn(i);
        });
    for (auto &x : th) x.join();
}

// table[m] = cos(pi m / (2n)), m = 0 .. 4n-1
std::vector<double> cos_table(int n) {
    std::vector<double> t((size_t)4 * n);
    for (int m = 0; m < 4 * n; ++m) t[m] = std::cos(kPi * (double)m / (2.0 * n));
    return t;
}
}  // namespace

std::vector<double> cheb_nodes(double lo, double hi, int n) {
    double sigma, tau;
    scale_shift(lo, hi, &sigma, &tau);
    std::vector<double> x(n);
    for (int k = 0; k < n; ++k) x[k] = std::cos(kPi * (k + 0.5) / n) / sigma + tau;
    return x;
}

std::vector<double> cheb_coeffs_from_samples(const std::vector<double> &fx) {
    const int n = (int)fx.size();
    std::vector<double> c(n, 0.0);
    if (n == 0) return c;
    const std::vector<double> tab = cos_table(n);
    const int period = 4 * n;
    parallel_for(n, [&](int j) {
        // cos(pi j (2k+1) / (2n)) = tab[j (2k+1) mod 4n]
        int idx = j % period;          // k = 0
        const int stepj = (2 * j) % period;
        double s = 0.0;
        for (int k = 0; k < n; ++k) {
            s += fx[k] * tab[idx];
            idx += stepj;
            if (idx >= period) idx -= period;
        }
        c[j] = 2.0 / n * s;
    });
    return c;
}

std::vector<double> cheb_coeffs(const Fn &f, double lo, double hi, int n) {
    const std::vector<double> x = cheb_nodes(lo, hi, n);
    std::vector<double> fx(n);
    for (int k = 0; k < n; ++k) fx[k] = f(x[k]);
    return cheb_coeffs_from_samples(fx);
}

double cheb_eval(const std::vector<double> &c, int m, double x) {
    // Clenshaw: b_k = c_k + 2 x b_{k+1} - b_{k+2}; p = b_0 - x b_1 - c_0/2
    double b1 = 0.0, b2 = 0.0;
    for (int k = m - 1; k >= 1; --k) {
        const double b0 = c[k] + 2.0 * x * b1 - b2;
        b2 = b1;
        b1 = b0;
    }
    return 0.5 * c[0] + x * b1 - b2;
}

double fit_error(const Fn &f, double lo, double hi, int m, int npts) {
    if (npts <= 0) npts = fit_points(m);
    const std::vector<double> c = cheb_coeffs(f, lo, hi, m);
    double sigma, tau;
    scale_shift(lo, hi, &sigma, &tau);
    std::vector<double> e((size_t)npts);
    parallel_for(npts, [&](int i) {
        const double xs = std::cos(kPi * (double)i / (npts - 1));
        const double x = xs / sigma + tau;
        e[i] = std::fabs(cheb_eval(c, m, xs) - f(x));
    });
    double err = 0.0;
    for (double v : e) err = std::max(err, v);
    return err;
}

int degree(const Fn &f, double lo, double hi, double tol, int step, int m_max, int npts) {
    int m = step;
    int last_bad = 0;
    while (true) {
        if (fit_error(f, lo, hi, m, npts) < tol) break;
        last_bad = m;
        if (m >= m_max) return -1;
        m = std::min(2 * m, m_max);
    }
    // smallest good multiple of step in (last_bad, m]
    int a = last_bad / step, b = m / step;  // a bad (or 0), b good
    while (b - a > 1) {
        const int mid = (a + b) / 2;
        if (fit_error(f, lo, hi, mid * step, npts) < tol)
            b = mid;
        else
            a = mid;
    }
    return b * step;
}

void CountFunction::init(const std::vector<double> &t, double lo_, double hi_, double kT_,
                         int smearing_) {
    lo = lo_;
    hi = hi_;
    kT = kT_;
    smearing = smearing_;
    const int n = (int)t.size();
    x = cheb_nodes(lo, hi, n);
    g.assign(n, 0.0);
    const std::vector<double> tab = cos_table(n);
    const int period = 4 * n;
    parallel_for(n, [&](int m) {
        // cos(j theta_m) = cos(pi j (2m+1)/(2n)) = tab[j (2m+1) mod 4n]
        double s = 0.5 * t[0];
        int idx = 0;
        const int stepm = (2 * m + 1) % period;
        for (int j = 1; j < n; ++j) {
            idx += stepm;
            if (idx >= period) idx -= period;
            s += t[j] * tab[idx];
        }
        g[m] = s;
    });
    cum.assign(n + 1, 0.0);
    for (int m = 0; m < n; ++m) cum[m + 1] = cum[m] + g[m];
}

double CountFunction::operator()(double mu) const {
    const int n = (int)g.size();
    double s = 0.0;
    for (int m = 0; m < n; ++m) {
        const double f = smearing == 0 ? occ_erfc(x[m], mu, kT) : occ_fd(x[m], mu, kT);
        s += f * g[m];
    }
    return 2.0 / n * s;
}

double CountFunction::local(double mu) const {
    // x is descending: nodes with x_m > mu + cut*kT are empty, below mu - cut*kT full
    const int n = (int)g.size();
    const double cut = (smearing == 0 ? 10.0 : 40.0) * kT;
    // first index with x_m <= mu + cut
    int a = (int)(std::upper_bound(x.begin(), x.end(), mu + cut, std::greater<double>()) - x.begin());
    // first index with x_m < mu - cut
    int b = (int)(std::upper_bound(x.begin(), x.end(), mu - cut, std::greater<double>()) - x.begin());
    while (b < n && x[b] >= mu - cut) ++b;
    double s = cum[n] - cum[b];  // fully occupied nodes
    for (int m = a; m < b; ++m) {
        const double f = smearing == 0 ? occ_erfc(x[m], mu, kT) : occ_fd(x[m], mu, kT);
        s += f * g[m];
    }
    return 2.0 / n * s;
}

bool bisect_mu(const CountFunction &N, double target, double tol_n, double a, double b,
               double *mu, int *iters) {
    double na = N(a), nb = N(b);
    int it = 0;
    if (!(na <= target && target <= nb)) {
        *iters = 0;
        return false;
    }
    double mid = 0.5 * (a + b);
    while (it < 200) {
        ++it;
        mid = 0.5 * (a + b);
        const double nm = N(mid);
        if (std::fabs(nm - target) <= tol_n || (b - a) <= 1e-13) break;
        if (nm < target)
            a = mid;
        else
            b = mid;
    }
    *mu = mid;
    *iters = it;
    return true;
}

std::vector<double> eigenvalues(const CountFunction &N, double e_lo, double e_hi, double tol_e) {
    std::vector<double> out;
    const double n_lo = N.local(e_lo), n_hi = N.local(e_hi);
    const long first = (long)std::floor(n_lo + 0.5) + 1;
    const long last = (long)std::floor(n_hi + 0.5);
    if (last < first) return out;
    // tabulate N on a grid of kT/8 and refine each crossing by bisection
    const double h = N.kT / 8.0;
    const long ng = std::max<long>(2, (long)std::ceil((e_hi - e_lo) / h) + 1);
    std::vector<double> grid(ng), val(ng);
    for (long i = 0; i < ng; ++i) {
        grid[i] = (i == ng - 1) ? e_hi : e_lo + h * i;
        val[i] = N.local(grid[i]);
    }
    long cell = 0;
    for (long Nn = first; Nn <= last; ++Nn) {
        const double target = Nn - 0.5;
        if (!(n_lo < target && target < n_hi)) continue;
        while (cell + 1 < ng - 1 && val[cell + 1] < target) ++cell;
        double a = grid[cell], b = grid[cell + 1];
        while (b - a > tol_e) {
            const double mid = 0.5 * (a + b);
            if (N.local(mid) < target)
                a = mid;
            else
                b = mid;
        }
        out.push_back(0.5 * (a + b));
    }
    return out;
}

double penalty_trace(const std::vector<double> &t, double alpha, double *fit_err) {
    const int n = (int)t.size();
    Fn fp = [alpha](double x) { return std::exp(alpha * (x + 1.0)) - std::exp(-alpha * (x - 1.0)); };
    const std::vector<double> c = cheb_coeffs(fp, -1.0, 1.0, n);
    double s = 0.5 * c[0] * t[0];
    for (int j = 1; j < n; ++j) s += c[j] * t[j];
    if (fit_err) *fit_err = fit_error(fp, -1.0, 1.0, std::min(n, 1024));
    return s;
}

int penalty_degree(long long n_rows) {
    const double alpha = -200.0;
    Fn fp = [alpha](double x) { return std::exp(alpha * (x + 1.0)) - std::exp(-alpha * (x - 1.0)); };
    const int m = degree(fp, -1.0, 1.0, 0.1 / (double)std::max(n_rows, 1LL), 8, 1024);
    return m < 0 ? 1024 : m;
}

BoundsCheck bounds_check(const std::vector<double> &t, long long n_rows) {
    BoundsCheck r;
    bool grows = false;
    for (double v : t)
        if (!std::isfinite(v) || std::fabs(v) > 1.01 * (double)n_rows) grows = true;
    if (grows) {
        // the moments' sign pattern over the last 16 terms: alternating for
        // an eigenvalue below the lower bound, one sign above the upper one
        r.ok = false;
        double alt = 0.0, same = 0.0;
        const size_t k0 = t.size() > 16 ? t.size() - 16 : 0;
        for (size_t k = k0; k < t.size(); ++k) {
            double v = t[k];
            if (std::isnan(v)) v = 0.0;
            if (std::isinf(v)) v = v > 0 ? 1e300 : -1e300;
            alt += (k % 2 == 0) ? v : -v;
            same += v;
        }
        r.side = std::fabs(alt) > std::fabs(same) ? -1 : 1;
        return r;
    }
    double fit_err = 1.0;
    const double pen = penalty_trace(t, -200.0, &fit_err);
    r.valid = fit_err * (double)n_rows < 0.1;
    if (r.valid) {
        r.penalty = pen;
        if (std::fabs(pen) > 0.5) {
            r.ok = false;
            r.side = pen > 0 ? -1 : 1;
        }
    }
    return r;
}

namespace {
// number of eigenvalues of T below x (Sturm sequence)
int sturm_count(const std::vector<double> &a, const std::vector<double> &b, double x) {
    int cnt = 0;
    double q = a[0] - x;
    if (q < 0) ++cnt;
    for (size_t i = 1; i < a.size(); ++i) {
        const double qq = (q == 0.0) ? 1e-300 : q;
        q = a[i] - x - b[i - 1] * b[i - 1] / qq;
        if (q < 0) ++cnt;
    }
    return cnt;
}

double kth_eig(const std::vector<double> &a, const std::vector<double> &b, int k) {
    // k-th smallest (0-based); Gershgorin interval of T
    double lo = 1e300, hi = -1e300;
    const size_t m = a.size();
    for (size_t i = 0; i < m; ++i) {
        double r = 0.0;
        if (i > 0) r += std::fabs(b[i - 1]);
        if (i + 1 < m) r += std::fabs(b[i]);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(lo) + std::fabs(hi));
         ++it) {
        const double mid = 0.5 * (lo + hi);
        if (sturm_count(a, b, mid) > k)
            hi = mid;
        else
            lo = mid;
    }
    return 0.5 * (lo + hi);
}

// last component of the normalised eigenvector for eigenvalue th (inverse iteration)
double last_component(const std::vector<double> &a, const std::vector<double> &b, double th) {
    const size_t m = a.size();
    if (m == 1) return 1.0;
    std::vector<double> v(m, 1.0 / std::sqrt((double)m)), y(m);
    const double shift = th + 1e-12 * std::max(1.0, std::fabs(th));
    for (int it = 0; it < 4; ++it) {
        // solve (T - shift I) y = v with Gaussian elimination (partial pivoting
        // is unnecessary for the tiny perturbation used as shift's safeguard)
        std::vector<double> d(m), u(m), l(m), rhs(v);
        for (size_t i = 0; i < m; ++i) d[i] = a[i] - shift;
        for (size_t i = 0; i + 1 < m; ++i) u[i] = b[i];
        for (size_t i = 1; i < m; ++i) {
            const double piv = (d[i - 1] == 0.0) ? 1e-300 : d[i - 1];
            const double f = b[i - 1] / piv;
            d[i] -= f * u[i - 1];
            rhs[i] -= f * rhs[i - 1];
        }
        y[m - 1] = rhs[m - 1] / ((d[m - 1] == 0.0) ? 1e-300 : d[m - 1]);
        for (size_t i = m - 1; i-- > 0;) y[i] = (rhs[i] - u[i] * y[i + 1]) / ((d[i] == 0.0) ? 1e-300 : d[i]);
        double nrm = 0.0;
        for (size_t i = 0; i < m; ++i) nrm += y[i] * y[i];
        nrm = std::sqrt(nrm);
        if (!(nrm > 0) || !std::isfinite(nrm)) break;
        for (size_t i = 0; i < m; ++i) v[i] = y[i] / nrm;
    }
    return v[m - 1];
}
}  // namespace

void tridiag_extremes(const std::vector<double> &alpha, const std::vector<double> &beta,
                      double beta_last, double *tmin, double *tmax, double *rmin, double *rmax) {
    const int m = (int)alpha.size();
    *tmin = kth_eig(alpha, beta, 0);
    *tmax = kth_eig(alpha, beta, m - 1);
    *rmin = std::fabs(beta_last * last_component(alpha, beta, *tmin));
    *rmax = std::fabs(beta_last * last_component(alpha, beta, *tmax));
}

}  // namespace hostmath
}  // namespace chess
