// Test shim: the library's host tables (Fejer rules, differentiation
// matrices) as flat arrays.  Built with the host compiler by the CPU tests.
#include <cstddef>
#include <vector>

#include "rules.hpp"

extern "C" void fejer_rule_c(int n, double* x, double* w) {
    std::vector<double> xv, wv;
    cbie::fejer_rule(n, xv, wv);
    for (int i = 0; i < n; ++i) { x[i] = xv[i]; w[i] = wv[i]; }
}

// returns the number of entries written (sum of q^2 for q = 1..qmax)
extern "C" int cheb_diff_matrices_c(int qmax, double* out, int cap) {
    std::vector<double> dm;
    cbie::cheb_diff_matrices(qmax, dm);
    if ((int)dm.size() > cap) return -1;
    for (size_t i = 0; i < dm.size(); ++i) out[i] = dm[i];
    return (int)dm.size();
}
