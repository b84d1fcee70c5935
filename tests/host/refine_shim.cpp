// Test shim: the library's stationary refinement control flow over host
// vectors, with a dense operator A and a dense approximate inverse M
// (column-major, interleaved real/imaginary parts), nrhs columns.  Built
// with the host compiler by the CPU tests.
#include <complex>
#include <vector>

#include "refine.hpp"

namespace {
using cd = std::complex<double>;
struct DenseOps {
    int n, nrhs;
    const cd *A, *M, *B;
    std::vector<cd> x, r;
    int residuals = 0;
    void mv(const cd* Mat, const cd* v, cd* y) {
        for (int i = 0; i < n; ++i) y[i] = 0.0;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) y[i] += Mat[(size_t)j * n + i] * v[j];
    }
    void ratios(std::vector<double>& q) {
        ++residuals;
        q.assign(nrhs, 0.0);
        std::vector<cd> ax(n);
        for (int c = 0; c < nrhs; ++c) {
            mv(A, &x[(size_t)c * n], ax.data());
            double rn = 0, bn = 0;
            for (int i = 0; i < n; ++i) {
                const cd b = B[(size_t)c * n + i];
                r[(size_t)c * n + i] = b - ax[i];
                rn += std::norm(r[(size_t)c * n + i]);
                bn += std::norm(b);
            }
            q[c] = std::sqrt(rn / (bn > 1e-300 ? bn : 1e-300));
        }
    }
    void correct() {
        std::vector<cd> d(n);
        for (int c = 0; c < nrhs; ++c) {
            mv(M, &r[(size_t)c * n], d.data());
            for (int i = 0; i < n; ++i) x[(size_t)c * n + i] += d[i];
        }
    }
};
}  // namespace

// x = M b, then refine; info: [corrections, residual evaluations, converged, nonfinite]
extern "C" void refine_dense(int n, int nrhs, const double* A, const double* M, const double* B, double* x,
                             double tol, int maxit, int* info, double* worst) {
    DenseOps op{n, nrhs, reinterpret_cast<const cd*>(A), reinterpret_cast<const cd*>(M),
                reinterpret_cast<const cd*>(B), std::vector<cd>((size_t)n * nrhs), std::vector<cd>((size_t)n * nrhs)};
    for (int c = 0; c < nrhs; ++c) op.mv(op.M, op.B + (size_t)c * n, &op.x[(size_t)c * n]);
    const cbie::RefineResult res = cbie::refine(op, tol, maxit);
    for (size_t e = 0; e < op.x.size(); ++e) reinterpret_cast<cd*>(x)[e] = op.x[e];
    info[0] = res.corrections;
    info[1] = op.residuals;
    info[2] = res.converged ? 1 : 0;
    info[3] = res.nonfinite ? 1 : 0;
    *worst = res.worst;
}
