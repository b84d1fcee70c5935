// Test shim: the library's GMRES refinement over host vectors, with a dense
// operator A and a dense approximate inverse M (column-major, interleaved
// real/imaginary parts).  Built with the host compiler by the CPU tests.
#include <complex>
#include <vector>

#include "gmres.hpp"

namespace {
using cd = std::complex<double>;
struct DenseOps {
    using Vec = std::vector<cd>;
    int n;
    const cd* A;
    const cd* M;
    int applies = 0, preconds = 0;
    Vec make() { return Vec(n, cd(0.0)); }
    static void mv(int n, const cd* Mat, const Vec& x, Vec& y) {
        for (int i = 0; i < n; ++i) y[i] = 0.0;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) y[i] += Mat[(size_t)j * n + i] * x[j];
    }
    void apply(const Vec& x, Vec& y) { ++applies; mv(n, A, x, y); }
    void precond(const Vec& r, Vec& z) { ++preconds; mv(n, M, r, z); }
    cd dot(const Vec& x, const Vec& y) {
        cd s = 0.0;
        for (int i = 0; i < n; ++i) s += std::conj(x[i]) * y[i];
        return s;
    }
    double nrm2(const Vec& x) { return std::sqrt(std::real(dot(x, x))); }
    void axpy(cd a, const Vec& x, Vec& y) { for (int i = 0; i < n; ++i) y[i] += a * x[i]; }
    void scal(cd a, Vec& x) { for (auto& v : x) v *= a; }
    void copy(const Vec& x, Vec& y) { y = x; }
};
}  // namespace

// info: [iterations, cycles, applications of A, applications of M]
extern "C" int gmres_dense(int n, const double* A, const double* M, const double* b, double* x, double tol,
                           int restart, int max_iter, int* info, double* rel_residual) {
    DenseOps op{n, reinterpret_cast<const cd*>(A), reinterpret_cast<const cd*>(M)};
    std::vector<cd> bv(reinterpret_cast<const cd*>(b), reinterpret_cast<const cd*>(b) + n);
    std::vector<cd> xv(reinterpret_cast<const cd*>(x), reinterpret_cast<const cd*>(x) + n);
    const cbie::GmresResult r = cbie::gmres_ir(op, bv, xv, tol, restart, max_iter);
    for (int i = 0; i < n; ++i) reinterpret_cast<cd*>(x)[i] = xv[i];
    info[0] = r.iterations;
    info[1] = r.cycles;
    info[2] = op.applies;
    info[3] = op.preconds;
    *rel_residual = r.rel_residual;
    return r.converged ? 1 : 0;
}
