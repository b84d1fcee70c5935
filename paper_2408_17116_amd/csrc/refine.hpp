// Stationary iterative refinement in FP64 around a low-precision
// factorization: x = M b, then repeat r = b - A x, x += M r, where A is the
// stored FP64 operator and M the substitutions with the complex64 H-LU.
//
// Host control flow only; the vector work comes from Ops, so the library
// runs it over device vectors and the tests over host vectors.  Ops provides
//   void ratios(std::vector<double>& q);  r = b - A x and q_j = ||r_j|| / ||b_j||
//                                         per right-hand side j
//   void correct();                       x += M r (the r of the last ratios)
//
// Semantics.  maxit = 0 asks for the plain substitution: no residual is
// formed and the result counts as converged.  Otherwise the residual is
// checked before every correction and once more after the last one, so a
// correction that reaches the tolerance is always seen: at most maxit
// corrections and maxit + 1 residual evaluations.  A non-finite ratio (an
// overflowing or NaN factorization) is a failure, never convergence.
#pragma once
#include <cmath>
#include <vector>

namespace cbie {

struct RefineResult {
    int corrections = 0;      // sweeps x += M r taken
    double worst = 0.0;       // largest ||r_j|| / ||b_j|| at the last check (+inf if non-finite)
    bool converged = false;
    bool nonfinite = false;
};

// Largest ratio; +inf as soon as one is not finite.
inline double worst_ratio(const std::vector<double>& q) {
    double w = 0.0;
    for (double v : q) {
        if (!std::isfinite(v)) return INFINITY;
        w = v > w ? v : w;
    }
    return w;
}

template <typename Ops> RefineResult refine(Ops& op, double tol, int maxit) {
    RefineResult out;
    if (maxit <= 0) {
        out.converged = true;
        return out;
    }
    std::vector<double> q;
    for (;;) {
        op.ratios(q);
        out.worst = worst_ratio(q);
        if (!std::isfinite(out.worst)) {
            out.nonfinite = true;
            return out;
        }
        if (out.worst <= tol) {
            out.converged = true;
            return out;
        }
        if (out.corrections >= maxit) return out;
        op.correct();
        ++out.corrections;
    }
}

}  // namespace cbie
