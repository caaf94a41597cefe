// Small dense fp64 linear algebra on the host for the a-posteriori
// certification (Prop. 3.7).  Column-major m x m matrices, leading dimension m.
#include "rgs_dense.hpp"

#include <algorithm>
#include <cfloat>
#include <cmath>

namespace rgs {
namespace dense {

namespace {

// sum_p a[p] b[p] over p < n in eight interleaved partial sums: independent
// chains keep the adders busy where one running sum waits on each add.
double dot(const double* a, const double* b, int n) {
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int p = 0;
    for (; p + 8 <= n; p += 8)
        for (int u = 0; u < 8; ++u) s[u] += a[p + u] * b[p + u];
    for (; p < n; ++p) s[p & 7] += a[p] * b[p];
    return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

}  // namespace

bool cholesky_upper(std::vector<double>& G, int m) {
    for (int j = 0; j < m; ++j) {
        double* gj = G.data() + (size_t)j * m;
        for (int i = 0; i < j; ++i) {
            const double* ti = G.data() + (size_t)i * m;
            gj[i] = (gj[i] - dot(ti, gj, i)) / ti[i];
        }
        const double d = gj[j] - dot(gj, gj, j);
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
        for (int i = j; i < m; ++i)
            if (!std::isfinite(A[i + (size_t)j * m])) return false;
    std::vector<double> d(m), e(std::max(m - 1, 0), 0.0), v(m), p(m);
    // Householder reduction on the lower triangle only: step j zeroes column j
    // below the subdiagonal and applies the reflector to both sides of the
    // trailing block (a symmetric rank-2 update of its lower triangle).
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
        const double vv = dot(v.data(), v.data(), r);
        e[j] = alpha;
        if (vv == 0.0) continue;
        const double tau = 2.0 / vv;
        double* B = A.data() + (size_t)(j + 1) * m + (j + 1);   // trailing block, leading dimension m
        // p = tau B v from the stored lower triangle: column c of it gives
        // p[c] (as a row of B, by symmetry) and adds to p[c+1..r)
        for (int i = 0; i < r; ++i) p[i] = 0.0;
        for (int c = 0; c < r; ++c) {
            const double* bc = B + (size_t)c * m;
            const double vc = v[c];
            p[c] += bc[c] * vc + dot(bc + c + 1, v.data() + c + 1, r - c - 1);
            for (int i = c + 1; i < r; ++i) p[i] += bc[i] * vc;
        }
        for (int i = 0; i < r; ++i) p[i] *= tau;
        const double K = 0.5 * tau * dot(p.data(), v.data(), r);
        for (int i = 0; i < r; ++i) p[i] -= K * v[i];   // w = p - K v
        for (int c = 0; c < r; ++c) {   // B -= v w^T + w v^T, lower triangle
            double* bc = B + (size_t)c * m;
            const double vc = v[c], wc = p[c];
            for (int i = c; i < r; ++i) bc[i] -= v[i] * wc + p[i] * vc;
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
