// Rank predictor: a fully connected 8 -> 64 -> 64 -> 1 ReLU network on the
// standardized geometric features of an admissible block, predicting the
// natural logarithm of its ACA rank.  Forward pass, gradient of the mean
// squared error by backpropagation, and Adam training, all in FP32.
//
// Parameter layout: W1 (64 x 8, row-major), b1 (64), W2 (64 x 64,
// row-major), b2 (64), W3 (64), b3 (1).
#include <cmath>
#include <vector>

#include "ctx.hpp"
#include "mlp.hpp"

namespace cbie {

constexpr int NI = kMlpIn, NH = kMlpHidden, NP = kMlpParams;
constexpr int OW1 = 0, OB1 = NH * NI, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH, OB3 = OW3 + NH;
static_assert(OB3 + 1 == NP, "parameter layout");

// ------------------------------------------------------------ forward
// One thread per sample; weights staged in LDS.
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ params, const float* __restrict__ mean,
                                                     const float* __restrict__ sdev, const float* __restrict__ X,
                                                     int64_t n, float* __restrict__ y) {
    __shared__ float P[NP];
    for (int e = threadIdx.x; e < NP; e += 256) P[e] = params[e];
    __syncthreads();
    const int64_t s = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (s >= n) return;
    float x[NI], h1[NH];
    for (int k = 0; k < NI; ++k) x[k] = (X[s * NI + k] - mean[k]) / sdev[k];
    for (int i = 0; i < NH; ++i) {
        float z = P[OB1 + i];
        for (int k = 0; k < NI; ++k) z = fmaf(P[OW1 + i * NI + k], x[k], z);
        h1[i] = fmaxf(z, 0.f);
    }
    float out = P[OB3];
    for (int j = 0; j < NH; ++j) {
        float z = P[OB2 + j];
        for (int i = 0; i < NH; ++i) z = fmaf(P[OW2 + j * NH + i], h1[i], z);
        out = fmaf(P[OW3 + j], fmaxf(z, 0.f), out);
    }
    y[s] = out;
}

// ----------------------------------------------------------- gradient
// One work-group accumulates, over samples taken 128 at a time, the gradient
// of sum_s (y_s - t_s)^2 / n_total into G (LDS).  P: parameters (LDS).
constexpr int CHUNK = 128;
struct MlpLds {
    float P[NP];
    float G[NP];
    // rows padded by one word: per-sample rows read by consecutive lanes
    // fall in different LDS banks
    float X[CHUNK][NI + 1];
    float H1[CHUNK][NH + 1];   // h1, then delta1
    float H2[CHUNK][NH + 1];   // h2
    float D2[CHUNK][NH + 1];   // delta2
    float dy[CHUNK];
    float red[4];
};

__device__ void mlp_chunk(MlpLds& L, const float* mean, const float* sdev, const float* X, const float* t,
                          const int* idx, int64_t base, int cn, float inv_n, float& loss_acc) {
    const int tid = threadIdx.x;
    // forward, one thread per sample
    if (tid < cn) {
        const int64_t s = idx ? (int64_t)idx[base + tid] : base + tid;
        float x[NI];
        for (int k = 0; k < NI; ++k) {
            x[k] = (X[s * NI + k] - mean[k]) / sdev[k];
            L.X[tid][k] = x[k];
        }
        for (int i = 0; i < NH; ++i) {
            float z = L.P[OB1 + i];
            for (int k = 0; k < NI; ++k) z = fmaf(L.P[OW1 + i * NI + k], x[k], z);
            L.H1[tid][i] = fmaxf(z, 0.f);
        }
        float out = L.P[OB3];
        for (int j = 0; j < NH; ++j) {
            float z = L.P[OB2 + j];
            for (int i = 0; i < NH; ++i) z = fmaf(L.P[OW2 + j * NH + i], L.H1[tid][i], z);
            const float h = fmaxf(z, 0.f);
            L.H2[tid][j] = h;
            out = fmaf(L.P[OW3 + j], h, out);
        }
        const float r = out - t[s];
        loss_acc += r * r * inv_n;
        L.dy[tid] = 2.f * r * inv_n;
    }
    __syncthreads();
    // delta2 per sample; d/dW3, d/db3 per output unit
    if (tid < cn) {
        for (int j = 0; j < NH; ++j) L.D2[tid][j] = L.H2[tid][j] > 0.f ? L.dy[tid] * L.P[OW3 + j] : 0.f;
    } else if (tid >= CHUNK && tid < CHUNK + NH + 1) {
        const int j = tid - CHUNK;
        float a = 0.f;
        if (j < NH)
            for (int q = 0; q < cn; ++q) a = fmaf(L.dy[q], L.H2[q][j], a);
        else
            for (int q = 0; q < cn; ++q) a += L.dy[q];
        L.G[j < NH ? OW3 + j : OB3] += a;
    }
    __syncthreads();
    // d/dW2 = sum_s delta2 h1^T, d/db2 = sum_s delta2
    for (int e = tid; e < NH * NH + NH; e += 256) {
        float a = 0.f;
        if (e < NH * NH) {
            const int j = e / NH, i = e % NH;
            for (int q = 0; q < cn; ++q) a = fmaf(L.D2[q][j], L.H1[q][i], a);
            L.G[OW2 + e] += a;
        } else {
            const int j = e - NH * NH;
            for (int q = 0; q < cn; ++q) a += L.D2[q][j];
            L.G[OB2 + j] += a;
        }
    }
    __syncthreads();
    // delta1 = (W2^T delta2) .* [h1 > 0], in place of h1
    if (tid < cn) {
        float d1[NH];
        for (int i = 0; i < NH; ++i) {
            float a = 0.f;
            for (int j = 0; j < NH; ++j) a = fmaf(L.P[OW2 + j * NH + i], L.D2[tid][j], a);
            d1[i] = L.H1[tid][i] > 0.f ? a : 0.f;
        }
        for (int i = 0; i < NH; ++i) L.H1[tid][i] = d1[i];
    }
    __syncthreads();
    // d/dW1 = sum_s delta1 x^T, d/db1 = sum_s delta1
    for (int e = tid; e < NH * NI + NH; e += 256) {
        float a = 0.f;
        if (e < NH * NI) {
            const int i = e / NI, k = e % NI;
            for (int q = 0; q < cn; ++q) a = fmaf(L.H1[q][i], L.X[q][k], a);
            L.G[OW1 + e] += a;
        } else {
            const int i = e - NH * NI;
            for (int q = 0; q < cn; ++q) a += L.H1[q][i];
            L.G[OB1 + i] += a;
        }
    }
    __syncthreads();
}

__device__ float block_sum_f(float v, float* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ params, const float* __restrict__ mean,
                                                  const float* __restrict__ sdev, const float* __restrict__ X,
                                                  const float* __restrict__ t, int64_t n, float* __restrict__ grad,
                                                  float* __restrict__ loss) {
    __shared__ MlpLds L;
    for (int e = threadIdx.x; e < NP; e += 256) {
        L.P[e] = params[e];
        L.G[e] = 0.f;
    }
    __syncthreads();
    float la = 0.f;
    const float inv_n = 1.f / (float)n;
    for (int64_t b = 0; b < n; b += CHUNK)
        mlp_chunk(L, mean, sdev, X, t, nullptr, b, (int)min((int64_t)CHUNK, n - b), inv_n, la);
    for (int e = threadIdx.x; e < NP; e += 256) grad[e] = L.G[e];
    const float tot = block_sum_f(la, L.red);
    if (threadIdx.x == 0) loss[0] = tot;
}

// Adam training in one work-group: step s uses the samples
// order[s * batch, (s + 1) * batch); m, v: moment buffers (zeroed here).
__global__ __launch_bounds__(256) void k_mlp_train(float* __restrict__ params, const float* __restrict__ mean,
                                                   const float* __restrict__ sdev, const float* __restrict__ X,
                                                   const float* __restrict__ t, const int* __restrict__ order,
                                                   int64_t nsteps, int batch, float lr, float* __restrict__ m,
                                                   float* __restrict__ v, float* __restrict__ losses) {
    __shared__ MlpLds L;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int e = threadIdx.x; e < NP; e += 256) {
        L.P[e] = params[e];
        m[e] = 0.f;
        v[e] = 0.f;
    }
    float b1t = 1.f, b2t = 1.f;
    const float inv_n = 1.f / (float)batch;
    for (int64_t st = 0; st < nsteps; ++st) {
        for (int e = threadIdx.x; e < NP; e += 256) L.G[e] = 0.f;
        __syncthreads();
        float la = 0.f;
        for (int b = 0; b < batch; b += CHUNK)
            mlp_chunk(L, mean, sdev, X, t, order, st * (int64_t)batch + b, min(CHUNK, batch - b), inv_n, la);
        const float tot = block_sum_f(la, L.red);
        if (threadIdx.x == 0) losses[st] = tot;
        b1t *= b1;
        b2t *= b2;
        for (int e = threadIdx.x; e < NP; e += 256) {
            const float g = L.G[e];
            const float mm = b1 * m[e] + (1.f - b1) * g;
            const float vv = b2 * v[e] + (1.f - b2) * g * g;
            m[e] = mm;
            v[e] = vv;
            L.P[e] -= lr * (mm / (1.f - b1t)) / (sqrtf(vv / (1.f - b2t)) + eps);
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < NP; e += 256) params[e] = L.P[e];
}

void mlp_forward(hipStream_t s, const float* params, const float* mean, const float* sdev, const float* X, int64_t n,
                 float* y) {
    if (n <= 0) return;
    k_mlp_forward<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(params, mean, sdev, X, n, y);
    check_launch("k_mlp_forward");
}
void mlp_grad(hipStream_t s, const float* params, const float* mean, const float* sdev, const float* X, const float* t,
              int64_t n, float* grad, float* loss) {
    k_mlp_grad<<<1, 256, 0, s>>>(params, mean, sdev, X, t, n, grad, loss);
    check_launch("k_mlp_grad");
}
void mlp_train(hipStream_t s, float* params, const float* mean, const float* sdev, const float* X, const float* t,
               const int* order, int64_t nsteps, int batch, float lr, float* losses) {
    DBuf<float> mv;
    mv.alloc(2 * (size_t)NP);
    k_mlp_train<<<1, 256, 0, s>>>(params, mean, sdev, X, t, order, nsteps, batch, lr, mv.p, mv.p + NP, losses);
    check_launch("k_mlp_train");
    CBIE_HIP(hipStreamSynchronize(s));   // the moment buffers are released on return
}

// ------------------------------------------------------------ features
// Per admissible block (t, s) of an object with wavenumber k:
//   log m, log n (unknowns), k diam_t, k diam_s, k dist, max(diam)/dist,
//   log10(tol), k diam_t diam_s / dist
// (diam: bounding-box diagonal, dist: gap between the boxes).
void block_features(const Ctx& c, double tol, std::vector<float>& f) {
    const int nb = (int)c.tree.lr_blocks.size();
    f.assign((size_t)nb * NI, 0.f);
    for (int b = 0; b < nb; ++b) {
        const Block& B = c.tree.blocks[c.tree.lr_blocks[b]];
        const Cluster &T = c.tree.clusters[B.t], &S = c.tree.clusters[B.s];
        const double k = c.objs[T.obj].k0;
        double dt = 0, ds = 0, gap = 0;
        for (int d = 0; d < 3; ++d) {
            dt += (T.bmax[d] - T.bmin[d]) * (T.bmax[d] - T.bmin[d]);
            ds += (S.bmax[d] - S.bmin[d]) * (S.bmax[d] - S.bmin[d]);
            const double g = std::max({0.0, S.bmin[d] - T.bmax[d], T.bmin[d] - S.bmax[d]});
            gap += g * g;
        }
        dt = std::sqrt(dt);
        ds = std::sqrt(ds);
        gap = std::max(std::sqrt(gap), 1e-12);
        float* x = &f[(size_t)b * NI];
        x[0] = (float)std::log((double)T.nunk());
        x[1] = (float)std::log((double)S.nunk());
        x[2] = (float)(k * dt);
        x[3] = (float)(k * ds);
        x[4] = (float)(k * gap);
        x[5] = (float)(std::max(dt, ds) / gap);
        x[6] = (float)std::log10(tol);
        x[7] = (float)(k * dt * ds / gap);
    }
}

}  // namespace cbie
