// Small dense fp64 linear algebra on the host for the a-posteriori
// certification (Prop. 3.7): the m x m factors and eigenvalue extremes that
// follow the device products.  All matrices are column-major, m x m, leading
// dimension m.
#pragma once

#include <vector>

namespace rgs {
namespace dense {

// G = T^T T with T upper triangular and positive diagonal, in place (the
// strict lower part is zeroed).  False if a pivot is not positive and finite.
bool cholesky_upper(std::vector<double>& G, int m);

// Inverse of the upper-triangular T (back substitution per column).
std::vector<double> upper_inverse(const std::vector<double>& T, int m);

// Smallest and largest eigenvalues of the symmetric A (only its lower
// triangle is read): Householder reduction to tridiagonal form, then
// bisection on Sturm sequence counts.  False if A is not finite.
bool sym_eig_extremes(std::vector<double> A, int m, double& lmin, double& lmax);

}  // namespace dense
}  // namespace rgs
