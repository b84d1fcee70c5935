// Host construction of the quadrature and interpolation tables the kernels
// read (Sec. II-B: Fejer's first rule on the Chebyshev points, eqs. 11-13;
// derivatives of the interpolant for the N-Mueller surface divergence).
#pragma once
#include <vector>

namespace cbie {

// Fejer-1 rule of size n on [-1, 1], nodes ascending:
// x_l = -cos((2l+1) pi / (2n)), w_l = (2/n)[1 - 2 sum_{m=1}^{n/2} cos(2 m th_l)/(4m^2 - 1)].
void fejer_rule(int n, std::vector<double>& x, std::vector<double>& w);

// Differentiation matrices of the degree q-1 interpolant at the q Fejer
// points, for q = 1..qmax, row-major and concatenated (q at offset
// (q-1) q (2q-1) / 6): D[i][j] = ell_j'(x_i), from the barycentric weights
// lam_j = 1 / prod_{k != j} (x_j - x_k): D[i][j] = (lam_j / lam_i) / (x_i - x_j),
// D[i][i] = -sum_{j != i} D[i][j].
void cheb_diff_matrices(int qmax, std::vector<double>& dm);

}  // namespace cbie
