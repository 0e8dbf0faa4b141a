// MLP kernels of the learned setup: a matrix-core GEMM and the elementwise,
// loss and optimiser kernels around it (layout and conventions in mlp.h).
#include <hip/hip_runtime.h>

#include "kp_common.h"
#include "mlp.h"

namespace kp {

typedef float gfloatx4 __attribute__((ext_vector_type(4)));
typedef short gshortx4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ GEMM
// 256 threads, a 64 x 64 tile of C per workgroup, four waves of 32 x 32
// (2 x 2 matrix-core tiles of 16 x 16), K in steps of 16 through LDS.
// Matrix-core operand layout (16 x 16 output, lane l = 16 g + c):
//   FP32 16x16x4: A[row c][k g], B[k g][col c];
//   BF16 16x16x16: A[row c][k 4g + i], B[k 4g + i][col c], i = 0..3;
//   result acc[v] = C[row 4g + v][col c].
template <bool kBF16>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const float* A, int lda, int transA,
                                              const float* B, int ldb, int transB, float* C, int ldc,
                                              float alpha, float beta) {
    __shared__ float As[64][17];
    __shared__ float Bs[16][65];
    const int tid = threadIdx.x, l = tid & 63, wv = tid >> 6;
    const int g = l >> 4, c = l & 15;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
    gfloatx4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = gfloatx4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        for (int q = tid; q < 64 * 16; q += 256) {
            int mm, kk;
            if (transA) { kk = q / 64; mm = q % 64; } else { mm = q / 16; kk = q % 16; }
            const int gm = m0 + mm, gk = k0 + kk;
            float v = 0.f;
            if (gm < M && gk < K) v = transA ? A[(long)gk * lda + gm] : A[(long)gm * lda + gk];
            As[mm][kk] = v;
        }
        for (int q = tid; q < 16 * 64; q += 256) {
            int kk, nn;
            if (transB) { nn = q / 16; kk = q % 16; } else { kk = q / 64; nn = q % 64; }
            const int gk = k0 + kk, gn = n0 + nn;
            float v = 0.f;
            if (gk < K && gn < N) v = transB ? B[(long)gn * ldb + gk] : B[(long)gk * ldb + gn];
            Bs[kk][nn] = v;
        }
        __syncthreads();
        for (int i = 0; i < 2; ++i) {
            for (int j = 0; j < 2; ++j) {
                const int rb = wm + 16 * i, cb = wn + 16 * j;
                if (kBF16) {
                    gshortx4 a, b;
                    for (int t = 0; t < 4; ++t) {
                        a[t] = (short)f32_to_bf16(As[rb + c][4 * g + t]);
                        b[t] = (short)f32_to_bf16(Bs[4 * g + t][cb + c]);
                    }
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[i][j], 0, 0, 0);
                } else {
                    for (int ks = 0; ks < 16; ks += 4) {
                        const float a = As[rb + c][ks + g];
                        const float b = Bs[ks + g][cb + c];
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i][j], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm + 16 * i + 4 * g + v;
                const int col = n0 + wn + 16 * j + c;
                if (row < M && col < N) {
                    float o = alpha * acc[i][j][v];
                    if (beta != 0.f) o += beta * C[(long)row * ldc + col];
                    C[(long)row * ldc + col] = o;
                }
            }
}

hipError_t launch_gemm(hipStream_t s, int bf16, int M, int N, int K, const float* A, int lda,
                       int transA, const float* B, int ldb, int transB, float* C, int ldc,
                       float alpha, float beta) {
    if (M <= 0 || N <= 0) return hipSuccess;
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    if (bf16)
        hipLaunchKernelGGL(k_gemm<true>, grid, dim3(256), 0, s, M, N, K, A, lda, transA, B, ldb, transB,
                           C, ldc, alpha, beta);
    else
        hipLaunchKernelGGL(k_gemm<false>, grid, dim3(256), 0, s, M, N, K, A, lda, transA, B, ldb, transB,
                           C, ldc, alpha, beta);
    return hipGetLastError();
}

// ------------------------------------------------------------ elementwise
__device__ inline float silu_f(float z) { return z / (1.f + expf(-z)); }
__device__ inline float silu_grad_f(float z) {
    const float sg = 1.f / (1.f + expf(-z));
    return sg * (1.f + z * (1.f - sg));
}

static int grid_for(long count) {
    long g = (count + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

__global__ void k_bias_silu(long count, int cols, float* Z, const float* b, float* H) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
        const float z = Z[i] + b[i % cols];
        Z[i] = z;
        H[i] = silu_f(z);
    }
}
hipError_t launch_bias_silu(hipStream_t s, int rows, int cols, float* Z, const float* b, float* H) {
    const long count = (long)rows * cols;
    hipLaunchKernelGGL(k_bias_silu, dim3(grid_for(count)), dim3(256), 0, s, count, cols, Z, b, H);
    return hipGetLastError();
}

__global__ void k_bias(long count, int cols, float* Y, const float* b) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x)
        Y[i] += b[i % cols];
}
hipError_t launch_bias(hipStream_t s, int rows, int cols, float* Y, const float* b) {
    const long count = (long)rows * cols;
    hipLaunchKernelGGL(k_bias, dim3(grid_for(count)), dim3(256), 0, s, count, cols, Y, b);
    return hipGetLastError();
}

__global__ void k_silu_back(long count, float* G, const float* Z) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x)
        G[i] *= silu_grad_f(Z[i]);
}
hipError_t launch_silu_back(hipStream_t s, int rows, int cols, float* G, const float* Z) {
    const long count = (long)rows * cols;
    hipLaunchKernelGGL(k_silu_back, dim3(grid_for(count)), dim3(256), 0, s, count, G, Z);
    return hipGetLastError();
}

// one thread per column, rows summed in order
__global__ void k_colsum(int rows, int cols, const float* G, float* out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float a = 0.f;
    for (int r = 0; r < rows; ++r) a += G[(long)r * cols + c];
    out[c] = a;
}
hipError_t launch_colsum(hipStream_t s, int rows, int cols, const float* G, float* out) {
    hipLaunchKernelGGL(k_colsum, dim3((cols + 255) / 256), dim3(256), 0, s, rows, cols, G, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ loss
// One workgroup per row.  Per factor block b: yy_b, yt_b, tt_b; the cost of
// sign pattern p is sum_b (yy_b - 2 s_pb yt_b + tt_b); the smallest (first on
// ties) is taken.  dY = scale * 2 (y - s t), row_loss = scale * cost.
__global__ void __launch_bounds__(256) k_mlp_loss(int rows, int dim, int n, const float* Y, const float* T,
                                                  float* dY, float* row_loss, float scale) {
    __shared__ double red[4 * kMaxReduce];
    __shared__ float sgn[5];
    BlockTeam tm{red};
    const int nn = n * n;
    const int nb = dim == 3 ? 5 : 4;
    const int O = nb * nn;
    const int np = dim == 3 ? 8 : 4;
    for (int r = blockIdx.x; r < rows; r += gridDim.x) {
        const float* y = Y + (long)r * O;
        const float* t = T + (long)r * O;
        double acc[15];
        for (int q = 0; q < 15; ++q) acc[q] = 0.0;
        for (int b = 0; b < nb; ++b)
            for (int i = threadIdx.x; i < nn; i += blockDim.x) {
                const double yv = y[b * nn + i], tv = t[b * nn + i];
                acc[3 * b] += yv * yv;
                acc[3 * b + 1] += yv * tv;
                acc[3 * b + 2] += tv * tv;
            }
        tm.sum_many(acc, 3 * nb);
        if (threadIdx.x == 0) {
            double best = 0.0;
            int bp = 0;
            for (int p = 0; p < np; ++p) {
                float s[5];
                if (dim == 3) {
                    const float s0 = (p & 4) ? -1.f : 1.f, s1 = (p & 2) ? -1.f : 1.f, s2 = (p & 1) ? -1.f : 1.f;
                    s[0] = s0; s[1] = s1; s[2] = s0 * s1; s[3] = s2; s[4] = s0 * s2;
                } else {
                    const float s1 = (p & 2) ? -1.f : 1.f, s2 = (p & 1) ? -1.f : 1.f;
                    s[0] = s1; s[1] = s1; s[2] = s2; s[3] = s2;
                }
                double cst = 0.0;
                for (int b = 0; b < nb; ++b) cst += acc[3 * b] - 2.0 * s[b] * acc[3 * b + 1] + acc[3 * b + 2];
                if (p == 0 || cst < best) {
                    best = cst;
                    bp = p;
                    for (int b = 0; b < nb; ++b) sgn[b] = s[b];
                }
            }
            (void)bp;
            row_loss[r] = (float)(scale * best);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < O; i += blockDim.x) dY[(long)r * O + i] = scale * 2.f * (y[i] - sgn[i / nn] * t[i]);
        __syncthreads();
    }
}
hipError_t launch_mlp_loss(hipStream_t s, int rows, int dim, int n, const float* Y, const float* T,
                           float* dY, float* row_loss, float scale) {
    if (rows <= 0) return hipSuccess;
    const int grid = rows < 65536 ? rows : 65536;
    hipLaunchKernelGGL(k_mlp_loss, dim3(grid), dim3(256), 0, s, rows, dim, n, Y, T, dY, row_loss, scale);
    return hipGetLastError();
}

// one workgroup: out[0] (+)= sum v (per-thread partials in order, then the waves)
__global__ void __launch_bounds__(256) k_sum(int count, const float* v, float* out, int accumulate) {
    __shared__ double red[4 * kMaxReduce];
    BlockTeam tm{red};
    double a = 0.0;
    for (int i = threadIdx.x; i < count; i += blockDim.x) a += v[i];
    a = tm.sum(a);
    if (threadIdx.x == 0) out[0] = accumulate ? (float)(out[0] + a) : (float)a;
}
hipError_t launch_sum(hipStream_t s, int count, const float* v, float* out, int accumulate) {
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, count, v, out, accumulate);
    return hipGetLastError();
}

// Adam (Kingma & Ba): c1 = 1 - beta1^t, c2 = 1 - beta2^t
__global__ void k_adam(long count, float* p, const float* g, float* m, float* v, float lr, float beta1,
                       float beta2, float eps, float c1, float c2) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = beta1 * m[i] + (1.f - beta1) * gi;
        const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}
hipError_t launch_adam(hipStream_t s, long count, float* p, const float* g, float* m, float* v,
                       float lr, float beta1, float beta2, float eps, float c1, float c2) {
    hipLaunchKernelGGL(k_adam, dim3(grid_for(count)), dim3(256), 0, s, count, p, g, m, v, lr, beta1, beta2,
                       eps, c1, c2);
    return hipGetLastError();
}

// ------------------------------------------------------ data preparation
// features: beta_x, beta_y, beta_z (0 in 2D), log10 nu, tau, alpha, sin phi,
// cos phi, c = 1 + alpha sin(pi x y [z] + phi) at four reference points
__global__ void k_mlp_features(int64_t E, int dim, const double* params, float* X) {
    const double pts[4][3] = {{0.25, 0.25, 0.25}, {0.75, 0.25, 0.75}, {0.25, 0.75, 0.75}, {0.75, 0.75, 0.25}};
    const double pi = 3.14159265358979323846;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
        const double* r = params + e * kRecLen;
        float* x = X + e * kMlpIn;
        x[0] = (float)r[0];
        x[1] = (float)r[1];
        x[2] = dim == 3 ? (float)r[2] : 0.f;
        x[3] = (float)log10(r[3]);
        x[4] = (float)r[6];
        x[5] = (float)r[4];
        x[6] = (float)sin(r[5]);
        x[7] = (float)cos(r[5]);
        for (int q = 0; q < 4; ++q) {
            const double prod = dim == 3 ? pts[q][0] * pts[q][1] * pts[q][2] : pts[q][0] * pts[q][1];
            x[8 + q] = (float)(1.0 + r[4] * sin(pi * prod + r[5]));
        }
    }
}
hipError_t launch_mlp_features(hipStream_t s, int64_t E, int dim, const double* params, float* X) {
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_features, dim3(grid_for(E)), dim3(256), 0, s, E, dim, params, X);
    return hipGetLastError();
}

// one workgroup per column: mean, then the population standard deviation
// (1 where it is zero)
__global__ void __launch_bounds__(256) k_col_stats(int64_t E, int I, const float* X, float* mean, float* sd) {
    __shared__ double red[4 * kMaxReduce];
    BlockTeam tm{red};
    const int c = blockIdx.x;
    double a = 0.0;
    for (int64_t e = threadIdx.x; e < E; e += blockDim.x) a += X[e * I + c];
    const double mu = tm.sum(a) / (double)(E > 0 ? E : 1);
    double q = 0.0;
    for (int64_t e = threadIdx.x; e < E; e += blockDim.x) {
        const double d = X[e * I + c] - mu;
        q += d * d;
    }
    const double var = tm.sum(q) / (double)(E > 0 ? E : 1);
    if (threadIdx.x == 0) {
        mean[c] = (float)mu;
        sd[c] = var > 0.0 ? (float)sqrt(var) : 1.f;
    }
}
hipError_t launch_col_stats(hipStream_t s, int64_t E, int I, const float* X, float* mean, float* sd) {
    hipLaunchKernelGGL(k_col_stats, dim3(I), dim3(256), 0, s, E, I, X, mean, sd);
    return hipGetLastError();
}

__global__ void k_normalise(long count, int I, const float* X, const float* mean, const float* sd, float* Xn) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x)
        Xn[i] = (X[i] - mean[i % I]) / sd[i % I];
}
hipError_t launch_normalise(hipStream_t s, int64_t E, int I, const float* X, const float* mean,
                            const float* sd, float* Xn) {
    const long count = (long)E * I;
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_normalise, dim3(grid_for(count)), dim3(256), 0, s, count, I, X, mean, sd, Xn);
    return hipGetLastError();
}

// one workgroup per block: RMS of the block's entries over all elements (1 if zero)
__global__ void __launch_bounds__(256) k_block_scale(int64_t E, int nb, int nn, const double* F, float* scale) {
    __shared__ double red[4 * kMaxReduce];
    BlockTeam tm{red};
    const int b = blockIdx.x;
    const long total = E * (long)nn;
    double a = 0.0;
    for (long q = threadIdx.x; q < total; q += blockDim.x) {
        const long e = q / nn, i = q % nn;
        const double v = F[(e * nb + b) * nn + i];
        a += v * v;
    }
    a = tm.sum(a);
    if (threadIdx.x == 0) scale[b] = a > 0.0 ? (float)sqrt(a / (double)total) : 1.f;
}
hipError_t launch_block_scale(hipStream_t s, int64_t E, int nb, int nn, const double* F, float* scale) {
    hipLaunchKernelGGL(k_block_scale, dim3(nb), dim3(256), 0, s, E, nb, nn, F, scale);
    return hipGetLastError();
}

__global__ void k_scale_targets(long count, int nb, int nn, const double* F, const float* scale, float* T) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x)
        T[i] = (float)(F[i] / (double)scale[(i / nn) % nb]);
}
hipError_t launch_scale_targets(hipStream_t s, int64_t E, int nb, int nn, const double* F,
                                const float* scale, float* T) {
    const long count = (long)E * nb * nn;
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_targets, dim3(grid_for(count)), dim3(256), 0, s, count, nb, nn, F, scale, T);
    return hipGetLastError();
}

__global__ void k_decode(long count, int nb, int nn, const float* Y, const float* scale, double* F) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x)
        F[i] = (double)Y[i] * (double)scale[(i / nn) % nb];
}
hipError_t launch_decode(hipStream_t s, int64_t E, int nb, int nn, const float* Y, const float* scale,
                         double* F) {
    const long count = (long)E * nb * nn;
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_decode, dim3(grid_for(count)), dim3(256), 0, s, count, nb, nn, Y, scale, F);
    return hipGetLastError();
}

__global__ void k_gather(int rows, const int32_t* idx, const float* X, int a, float* Xb, const float* T,
                         int b, float* Tb) {
    const long cnt = (long)rows * (a + b);
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < cnt; q += (long)gridDim.x * blockDim.x) {
        const long r = q / (a + b);
        const int c = (int)(q % (a + b));
        const long src = idx[r];
        if (c < a)
            Xb[r * a + c] = X[src * a + c];
        else
            Tb[r * b + (c - a)] = T[src * b + (c - a)];
    }
}
hipError_t launch_gather(hipStream_t s, int rows, const int32_t* idx, const float* X, int a, float* Xb,
                         const float* T, int b, float* Tb) {
    const long cnt = (long)rows * (a + b);
    if (cnt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(cnt)), dim3(256), 0, s, rows, idx, X, a, Xb, T, b, Tb);
    return hipGetLastError();
}

}  // namespace kp
