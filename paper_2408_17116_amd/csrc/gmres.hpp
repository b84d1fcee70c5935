// Restarted GMRES in FP64 with the H-LU factorization as a right
// preconditioner (GMRES-based iterative refinement).  Plain refinement
// x += M (b - A x) contracts only while the factorization M, truncated at
// the compression tolerance and rounded to complex64, satisfies
// ||I - M A|| < 1; close to a resonance of the operator that fails.  GMRES
// on A M y = b, x = M y, needs only that the spectrum of A M is clustered
// (around 1, with the few outliers that the near-singular directions
// produce), so it converges where the stationary iteration cannot.
//
// Host orchestration only: the vectors and the operations on them come from
// Ops, so the same code runs over device vectors in the library and over
// host vectors in the tests.  Ops provides
//   using Vec = ...;                                  a vector (movable)
//   Vec make();                                       a zero vector
//   void apply(const Vec& x, Vec& y);                 y = A x   (FP64)
//   void precond(const Vec& r, Vec& z);               z = M r
//   std::complex<double> dot(const Vec& x, const Vec& y);   x^H y
//   double nrm2(const Vec& x);
//   void axpy(std::complex<double> a, const Vec& x, Vec& y); y += a x
//   void scal(std::complex<double> a, Vec& x);        x *= a
//   void copy(const Vec& x, Vec& y);                  y = x
// One right-hand side per call.
#pragma once
#include <cmath>
#include <complex>
#include <vector>

namespace cbie {

struct GmresResult {
    int iterations = 0;       // Krylov steps over all cycles
    int cycles = 0;           // restarts + 1
    double rel_residual = 0;  // ||b - A x|| / ||b|| recomputed at the end
    bool converged = false;
};

// x: initial guess on entry, solution on return.  Stops when the true
// residual ||b - A x|| <= tol ||b|| or after max_iter Krylov steps; each
// cycle builds at most `restart` basis vectors.
template <typename Ops>
GmresResult gmres_ir(Ops& op, const typename Ops::Vec& b, typename Ops::Vec& x, double tol, int restart,
                     int max_iter) {
    using cd = std::complex<double>;
    using Vec = typename Ops::Vec;
    GmresResult out;
    const double bn = op.nrm2(b);
    if (bn == 0.0) {
        op.scal(cd(0.0), x);
        out.converged = true;
        return out;
    }
    const int m = restart < 1 ? 1 : restart;
    Vec r = op.make(), w = op.make();
    std::vector<Vec> V, Z;   // Arnoldi basis and its preconditioned images
    V.reserve(m + 1);
    Z.reserve(m);
    for (int i = 0; i <= m; ++i) V.push_back(op.make());
    for (int i = 0; i < m; ++i) Z.push_back(op.make());
    std::vector<cd> H((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m);
    auto h = [&](int i, int j) -> cd& { return H[(size_t)j * (m + 1) + i]; };
    for (;;) {
        // true residual of the current iterate
        op.apply(x, r);
        op.scal(cd(-1.0), r);
        op.axpy(cd(1.0), b, r);
        const double beta = op.nrm2(r);
        out.rel_residual = beta / bn;
        if (out.rel_residual <= tol) {
            out.converged = true;
            return out;
        }
        if (out.iterations >= max_iter) return out;
        ++out.cycles;
        op.copy(r, V[0]);
        op.scal(cd(1.0 / beta), V[0]);
        for (auto& v : g) v = cd(0.0);
        g[0] = cd(beta);
        int k = 0;   // basis vectors built in this cycle
        for (int j = 0; j < m && out.iterations < max_iter; ++j) {
            op.precond(V[j], Z[j]);
            op.apply(Z[j], w);
            // modified Gram-Schmidt
            for (int i = 0; i <= j; ++i) {
                h(i, j) = op.dot(V[i], w);
                op.axpy(-h(i, j), V[i], w);
            }
            const double hn = op.nrm2(w);
            h(j + 1, j) = cd(hn);
            // earlier rotations on the new column
            for (int i = 0; i < j; ++i) {
                const cd a = h(i, j), c = h(i + 1, j);
                h(i, j) = cs[i] * a + sn[i] * c;
                h(i + 1, j) = -std::conj(sn[i]) * a + cs[i] * c;
            }
            // the rotation that zeroes h(j + 1, j)
            const cd a = h(j, j), c = h(j + 1, j);
            const double t = std::sqrt(std::norm(a) + std::norm(c));
            if (std::abs(a) == 0.0) {
                cs[j] = cd(0.0);
                sn[j] = cd(1.0);
                h(j, j) = c;
            } else {
                const cd ph = a / std::abs(a);
                cs[j] = cd(std::abs(a) / t);
                sn[j] = ph * std::conj(c) / t;
                h(j, j) = ph * t;
            }
            h(j + 1, j) = cd(0.0);
            g[j + 1] = -std::conj(sn[j]) * g[j];
            g[j] = cs[j] * g[j];
            ++out.iterations;
            k = j + 1;
            if (hn == 0.0 || std::abs(g[j + 1]) <= tol * bn) break;   // happy breakdown or converged
            op.copy(w, V[j + 1]);
            op.scal(cd(1.0 / hn), V[j + 1]);
        }
        // y = R^{-1} g, x += Z y
        std::vector<cd> y(k);
        for (int i = k - 1; i >= 0; --i) {
            cd s = g[i];
            for (int l = i + 1; l < k; ++l) s -= h(i, l) * y[l];
            y[i] = s / h(i, i);
        }
        for (int i = 0; i < k; ++i) op.axpy(y[i], Z[i], x);
    }
}

}  // namespace cbie
