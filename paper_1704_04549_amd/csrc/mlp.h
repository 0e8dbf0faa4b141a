// Learned setup: the model buffer layout and the MLP kernels' launchers.
//
// Network (not part of the paper; the paper's SVD stays the arbiter):
//   xn = (features - x_mean) / x_std            (12 features per element)
//   h1 = silu(W1 xn + b1), h2 = silu(W2 h1 + b2), y = W3 h2 + b3,
//   factors = y * (per-block scale)             (3D: A1,B1,C1,B2,C2; 2D: A1,B1,A2,B2)
// All weights are FP32, row-major (W1: H x I, W2: H x H, W3: O x H).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace kp {

constexpr int kMlpMagic = 0x4b504d4c;
constexpr int kMlpIn = 12;

// header: int32[64] = {magic, I, H, O, dim, n, nblocks, step, ...}; then FP32
// arrays, each 256-byte aligned: params (P), adam m (P), adam v (P),
// x_mean (I), x_std (I), yscale (nblocks).
struct MlpLayout {
    int I, H, O, nb;
    long P;
    size_t params, m, v, xmean, xstd, yscale, total;
};

inline size_t mlp_align(size_t x) { return (x + 255) / 256 * 256; }

inline bool mlp_layout(int dim, int n, int hidden, MlpLayout* L) {
    if ((dim != 2 && dim != 3) || n < 2 || n > 32 || hidden < 1 || hidden > 4096) return false;
    L->I = kMlpIn;
    L->H = hidden;
    L->nb = dim == 3 ? 5 : 4;
    L->O = L->nb * n * n;
    L->P = (long)L->H * L->I + L->H + (long)L->H * L->H + L->H + (long)L->O * L->H + L->O;
    size_t off = 256;
    L->params = off; off = mlp_align(off + L->P * sizeof(float));
    L->m = off; off = mlp_align(off + L->P * sizeof(float));
    L->v = off; off = mlp_align(off + L->P * sizeof(float));
    L->xmean = off; off = mlp_align(off + L->I * sizeof(float));
    L->xstd = off; off = mlp_align(off + L->I * sizeof(float));
    L->yscale = off; off = mlp_align(off + L->nb * sizeof(float));
    L->total = off;
    return true;
}

// parameter offsets (floats) inside the params array
struct MlpParams {
    long W1, b1, W2, b2, W3, b3;
};
inline MlpParams mlp_params(const MlpLayout& L) {
    MlpParams p;
    p.W1 = 0;
    p.b1 = p.W1 + (long)L.H * L.I;
    p.W2 = p.b1 + L.H;
    p.b2 = p.W2 + (long)L.H * L.H;
    p.W3 = p.b2 + L.H;
    p.b3 = p.W3 + (long)L.O * L.H;
    return p;
}

// C[M x N] = alpha * opA(A) opB(B) + beta * C, row-major; opA(A)[m][k] =
// transA ? A[k*lda + m] : A[m*lda + k] (likewise B).  bf16: operands rounded
// to bf16, FP32 accumulation.
hipError_t launch_gemm(hipStream_t s, int bf16, int M, int N, int K, const float* A, int lda,
                       int transA, const float* B, int ldb, int transB, float* C, int ldc,
                       float alpha, float beta);
// Z[r][c] += b[c]; H = silu(Z)
hipError_t launch_bias_silu(hipStream_t s, int rows, int cols, float* Z, const float* b, float* H);
// Y[r][c] += b[c]
hipError_t launch_bias(hipStream_t s, int rows, int cols, float* Y, const float* b);
// G[r][c] *= silu'(Z[r][c])
hipError_t launch_silu_back(hipStream_t s, int rows, int cols, float* G, const float* Z);
// out[c] = sum_r G[r][c] (fixed order)
hipError_t launch_colsum(hipStream_t s, int rows, int cols, const float* G, float* out);
// sign-minimised MSE of a batch: per-row loss into row_loss, gradient into dY
hipError_t launch_mlp_loss(hipStream_t s, int rows, int dim, int n, const float* Y, const float* T,
                           float* dY, float* row_loss, float scale);
// out[0] (+)= sum of v[0..count) in fixed order (one workgroup)
hipError_t launch_sum(hipStream_t s, int count, const float* v, float* out, int accumulate);
hipError_t launch_adam(hipStream_t s, long count, float* p, const float* g, float* m, float* v,
                       float lr, float beta1, float beta2, float eps, float c1, float c2);
// features of element records (FP64 [E][16]) -> raw FP32 [E][12]
hipError_t launch_mlp_features(hipStream_t s, int64_t E, int dim, const double* params, float* X);
// column mean and standard deviation of X [E][I] (one workgroup per column)
hipError_t launch_col_stats(hipStream_t s, int64_t E, int I, const float* X, float* mean, float* std);
// Xn = (X - mean) / std
hipError_t launch_normalise(hipStream_t s, int64_t E, int I, const float* X, const float* mean,
                            const float* std, float* Xn);
// per-block RMS of FP64 factors [E][nb][n^2] -> scale[nb] (one workgroup per block)
hipError_t launch_block_scale(hipStream_t s, int64_t E, int nb, int nn, const double* F, float* scale);
// T = F / scale (FP64 -> FP32)
hipError_t launch_scale_targets(hipStream_t s, int64_t E, int nb, int nn, const double* F,
                                const float* scale, float* T);
// F = Y * scale (FP32 -> FP64)
hipError_t launch_decode(hipStream_t s, int64_t E, int nb, int nn, const float* Y, const float* scale,
                         double* F);
// rows idx[i] of X (cols a) and T (cols b) into Xb, Tb
hipError_t launch_gather(hipStream_t s, int rows, const int32_t* idx, const float* X, int a, float* Xb,
                         const float* T, int b, float* Tb);

}  // namespace kp
