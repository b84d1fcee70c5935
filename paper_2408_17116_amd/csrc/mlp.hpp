// Rank predictor network (8 -> 64 -> 64 -> 1, ReLU): kernels and features.
#pragma once
#include <vector>

#include "common.hpp"

namespace cbie {

constexpr int kMlpIn = 8, kMlpHidden = 64;
constexpr int kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden + kMlpHidden + 1;

struct Ctx;
// y[i] = f(params; (X[i] - mean) / sdev), X: n x 8 row-major (device)
void mlp_forward(hipStream_t s, const float* params, const float* mean, const float* sdev, const float* X, int64_t n,
                 float* y);
// loss = mean (f(x_i) - t_i)^2 and its gradient (device)
void mlp_grad(hipStream_t s, const float* params, const float* mean, const float* sdev, const float* X, const float* t,
              int64_t n, float* grad, float* loss);
// Adam: step s on samples order[s * batch, (s + 1) * batch); params in place
void mlp_train(hipStream_t s, float* params, const float* mean, const float* sdev, const float* X, const float* t,
               const int* order, int64_t nsteps, int batch, float lr, float* losses);
// 8 features per admissible block, in low-rank block order (host)
void block_features(const Ctx& c, double tol, std::vector<float>& f);

}  // namespace cbie
