// Host construction of the quadrature and interpolation tables.
#include "rules.hpp"

#include <cmath>

namespace cbie {

void fejer_rule(int n, std::vector<double>& x, std::vector<double>& w) {
    x.resize(n);
    w.resize(n);
    for (int l = 0; l < n; ++l) {
        const double th = (2 * l + 1) * M_PI / (2.0 * n);
        x[l] = -std::cos(th);
        double s = 1.0;
        for (int m = 1; m <= n / 2; ++m) s -= 2.0 * std::cos(2 * m * th) / (4.0 * m * m - 1.0);
        w[l] = 2.0 / n * s;
    }
}

void cheb_diff_matrices(int qmax, std::vector<double>& dm) {
    dm.clear();
    std::vector<double> x, w;
    for (int q = 1; q <= qmax; ++q) {
        fejer_rule(q, x, w);
        std::vector<double> lam(q, 1.0);
        for (int j = 0; j < q; ++j)
            for (int k = 0; k < q; ++k)
                if (k != j) lam[j] /= (x[j] - x[k]);
        for (int i = 0; i < q; ++i) {
            double diag = 0.0;
            std::vector<double> row(q, 0.0);
            for (int j = 0; j < q; ++j)
                if (j != i) {
                    row[j] = (lam[j] / lam[i]) / (x[i] - x[j]);
                    diag -= row[j];
                }
            row[i] = diag;
            dm.insert(dm.end(), row.begin(), row.end());
        }
    }
}

}  // namespace cbie
