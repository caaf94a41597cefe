// Small dense fp64 linear algebra on the host for the a-posteriori
// certification (Prop. 3.7).  Column-major m x m matrices, leading dimension m.
#include "rgs_dense.hpp"

#include <algorithm>
#include <cfloat>
#include <cmath>

namespace rgs {
namespace dense {

bool cholesky_upper(std::vector<double>& G, int m) {
    for (int j = 0; j < m; ++j) {
        double* gj = G.data() + (size_t)j * m;
        for (int i = 0; i < j; ++i) {
            const double* ti = G.data() + (size_t)i * m;
            double s = gj[i];
            for (int p = 0; p < i; ++p) s -= ti[p] * gj[p];
            gj[i] = s / ti[i];
        }
        double d = gj[j];
        for (int p = 0; p < j; ++p) d -= gj[p] * gj[p];
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        gj[j] = std::sqrt(d);
        for (int i = j + 1; i < m; ++i) gj[i] = 0.0;
    }
    return true;
}

std::vector<double> upper_inverse(const std::vector<double>& T, int m) {
    std::vector<double> X((size_t)m * m, 0.0);
    for (int j = 0; j < m; ++j) {
        double* x = X.data() + (size_t)j * m;
        x[j] = 1.0;
        // column-oriented back substitution of T x = e_j
        for (int p = j; p >= 0; --p) {
            const double* tp = T.data() + (size_t)p * m;
            x[p] /= tp[p];
            const double xp = x[p];
            for (int i = 0; i < p; ++i) x[i] -= tp[i] * xp;
        }
    }
    return X;
}

namespace {

// Number of eigenvalues of the symmetric tridiagonal (d, e) below x.
int sturm_count(const std::vector<double>& d, const std::vector<double>& e2, double x, double pivmin) {
    int cnt = 0;
    double q = d[0] - x;
    if (std::fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++cnt;
    for (size_t i = 1; i < d.size(); ++i) {
        q = d[i] - x - e2[i - 1] / q;
        if (std::fabs(q) < pivmin) q = -pivmin;
        if (q < 0) ++cnt;
    }
    return cnt;
}

}  // namespace

bool sym_eig_extremes(std::vector<double> A, int m, double& lmin, double& lmax) {
    for (int j = 0; j < m; ++j)
        for (int i = j; i < m; ++i) {
            const double v = A[i + (size_t)j * m];
            if (!std::isfinite(v)) return false;
            A[j + (size_t)i * m] = v;   // mirror the lower triangle
        }
    std::vector<double> d(m), e(std::max(m - 1, 0), 0.0), v(m), p(m);
    // Householder reduction: step j zeroes column j below the subdiagonal and
    // applies the reflector to both sides of the trailing block.
    for (int j = 0; j + 2 < m; ++j) {
        const int r = m - j - 1;
        double* x = A.data() + (size_t)j * m + j + 1;
        double nrm = 0.0;
        for (int i = 0; i < r; ++i) nrm = std::hypot(nrm, x[i]);
        d[j] = A[j + (size_t)j * m];
        if (nrm == 0.0) {
            e[j] = 0.0;
            continue;
        }
        const double alpha = x[0] > 0 ? -nrm : nrm;
        for (int i = 0; i < r; ++i) v[i] = x[i];
        v[0] -= alpha;
        double vv = 0.0;
        for (int i = 0; i < r; ++i) vv += v[i] * v[i];
        e[j] = alpha;
        if (vv == 0.0) continue;
        const double tau = 2.0 / vv;
        double* B = A.data() + (size_t)(j + 1) * m + (j + 1);   // trailing block, leading dimension m
        for (int i = 0; i < r; ++i) p[i] = 0.0;
        for (int c = 0; c < r; ++c) {
            const double vc = tau * v[c];
            const double* bc = B + (size_t)c * m;
            for (int i = 0; i < r; ++i) p[i] += bc[i] * vc;
        }
        double pv = 0.0;
        for (int i = 0; i < r; ++i) pv += p[i] * v[i];
        const double K = 0.5 * tau * pv;
        for (int i = 0; i < r; ++i) p[i] -= K * v[i];   // w = p - K v
        for (int c = 0; c < r; ++c) {
            double* bc = B + (size_t)c * m;
            const double vc = v[c], wc = p[c];
            for (int i = 0; i < r; ++i) bc[i] -= v[i] * wc + p[i] * vc;
        }
    }
    if (m >= 2) {
        d[m - 2] = A[(m - 2) + (size_t)(m - 2) * m];
        e[m - 2] = A[(m - 1) + (size_t)(m - 2) * m];
    }
    d[m - 1] = A[(m - 1) + (size_t)(m - 1) * m];

    // Gershgorin interval, then bisection for the first and the last eigenvalue
    std::vector<double> e2(e.size());
    double lo = INFINITY, hi = -INFINITY, emax2 = 0.0;
    for (int i = 0; i < m; ++i) {
        const double off = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(e[i]) : 0.0);
        lo = std::min(lo, d[i] - off);
        hi = std::max(hi, d[i] + off);
    }
    for (size_t i = 0; i < e.size(); ++i) {
        e2[i] = e[i] * e[i];
        emax2 = std::max(emax2, e2[i]);
    }
    if (!std::isfinite(lo) || !std::isfinite(hi)) return false;
    const double pivmin = DBL_MIN * std::max(1.0, emax2);
    const double span = std::max(std::fabs(lo), std::fabs(hi));
    lo -= 2.0 * DBL_EPSILON * span * m + pivmin;
    hi += 2.0 * DBL_EPSILON * span * m + pivmin;
    auto bisect = [&](int target) {   // smallest x with at least `target` eigenvalues below it
        double a = lo, b = hi;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (a + b);
            if (mid <= a || mid >= b) break;
            if (b - a <= 2.0 * DBL_EPSILON * std::max(std::fabs(a), std::fabs(b)) + pivmin) break;
            if (sturm_count(d, e2, mid, pivmin) >= target)
                b = mid;
            else
                a = mid;
        }
        return 0.5 * (a + b);
    };
    lmin = bisect(1);
    lmax = bisect(m);
    return true;
}

}  // namespace dense
}  // namespace rgs
