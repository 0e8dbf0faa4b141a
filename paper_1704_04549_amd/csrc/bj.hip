// Exact block Jacobi: batched LU with partial pivoting of the explicit
// diagonal blocks and the matching triangular solves.  The comparator of the
// paper (Sec. 5): O(N^3) form and O(N^2) apply per element, N = n^d.
//
// LU factors are stored row-major per element in place of the block (entry
// (i, j) at i*N + j; unit lower triangle below the diagonal, U on and above
// it); piv[e][k] is the row swapped with row k at step k (LAPACK order).
//
// Factorisation: one workgroup of four waves per element, right-looking and
// blocked by panels of nb columns.  A panel (the rows from its first column
// down, nb columns) is factored with partial pivoting in LDS; its row swaps
// are applied to the other columns; the block row right of the panel is
// solved with the panel's unit lower triangle; the trailing matrix is updated
// by A22 -= L21 U12 in 16 x 16 tiles on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64), L21 read from LDS, U12 and A22 from the element's
// matrix in HBM.  nb = 32 for N <= 568 (the panel, N x 33 doubles, fits in
// LDS), fewer columns above.
//
// Solves: one workgroup per (element, right-hand side), x in LDS.  The
// triangles are processed in blocks of 64 rows: the part left of (forward) or
// right of (backward) the diagonal block is a matrix-vector product whose rows
// are read with coalesced loads and reduced per wave; the 64 x 64 diagonal
// block is staged in LDS and swept by one wave, one row per lane.
#include <hip/hip_runtime.h>

#include "kp_common.h"
#include "krylov.h"

namespace kp {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr size_t kBjLdsMax = 150 * 1024;
constexpr int kBjNbMax = 32;

// panel width for N (the panel's LDS, N x (nb + 1) doubles, within kBjLdsMax)
__host__ __device__ inline int bj_panel_width(int N) {
    int nb = (int)(kBjLdsMax / (8 * (size_t)N)) - 1;
    if (nb > kBjNbMax) nb = kBjNbMax;
    if (nb < 1) nb = 1;
    return nb;
}

__device__ __forceinline__ void wave_argmax(double& v, int& i) {
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int oi = __shfl_xor(i, off, 64);
        if (ov > v || (ov == v && oi < i)) {
            v = ov;
            i = oi;
        }
    }
}

__device__ __forceinline__ double bj_wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ void __launch_bounds__(256) k_bj_factor(int64_t E, int N, int nb, const double* blocks,
                                                   double* lu, int32_t* piv, int32_t* status) {
    extern __shared__ double pan[];  // [N][nb + 1]
    __shared__ double vmax[4];
    __shared__ int imax[4];
    __shared__ int pk;
    __shared__ int pvt[kBjNbMax];   // the panel's pivot rows (panel-local)
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, c = l & 15;
    const int pp = nb + 1;
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        double* A = lu + e * (int64_t)N * N;
        int32_t* P = piv + e * (int64_t)N;
        if (blocks != lu) {
            const double* B = blocks + e * (int64_t)N * N;
            for (int64_t t = tid; t < (int64_t)N * N; t += blockDim.x) A[t] = B[t];
            __syncthreads();
        }
        int st = 0;
        for (int k0 = 0; k0 < N; k0 += nb) {
            const int nbk = N - k0 < nb ? N - k0 : nb;
            const int m = N - k0;
            // (a) the panel A[k0:N, k0:k0+nbk] into LDS, factored there
            for (int t = tid; t < m * nbk; t += blockDim.x) {
                const int i = t / nbk, j = t % nbk;
                pan[i * pp + j] = A[(int64_t)(k0 + i) * N + k0 + j];
            }
            __syncthreads();
            for (int j = 0; j < nbk; ++j) {
                double bv = -1.0;
                int bi = j;
                for (int i = j + tid; i < m; i += blockDim.x) {
                    const double v = fabs(pan[i * pp + j]);
                    if (v > bv) {
                        bv = v;
                        bi = i;
                    }
                }
                wave_argmax(bv, bi);
                if (l == 0) {
                    vmax[w] = bv;
                    imax[w] = bi;
                }
                __syncthreads();
                if (tid == 0) {
                    double b = vmax[0];
                    int ii = imax[0];
                    for (int q = 1; q < 4; ++q)
                        if (vmax[q] > b || (vmax[q] == b && imax[q] < ii)) {
                            b = vmax[q];
                            ii = imax[q];
                        }
                    pk = ii;
                    pvt[j] = ii;
                    P[k0 + j] = k0 + ii;
                }
                __syncthreads();
                const int p = pk;
                if (p != j)
                    for (int q = tid; q < nbk; q += blockDim.x) {
                        const double t = pan[j * pp + q];
                        pan[j * pp + q] = pan[p * pp + q];
                        pan[p * pp + q] = t;
                    }
                __syncthreads();
                const double pv = pan[j * pp + j];
                if (pv == 0.0) {
                    st |= 2;
                    continue;
                }
                const double ip = 1.0 / pv;
                for (int i = j + 1 + tid; i < m; i += blockDim.x) pan[i * pp + j] *= ip;
                __syncthreads();
                const int cols = nbk - j - 1;
                if (cols > 0)
                    for (int t = tid; t < (m - j - 1) * cols; t += blockDim.x) {
                        const int i = j + 1 + t / cols, q = j + 1 + t % cols;
                        pan[i * pp + q] -= pan[i * pp + j] * pan[j * pp + q];
                    }
                __syncthreads();
            }
            // (b) the panel back; its swaps applied to the columns left and right of it
            for (int t = tid; t < m * nbk; t += blockDim.x) {
                const int i = t / nbk, j = t % nbk;
                A[(int64_t)(k0 + i) * N + k0 + j] = pan[i * pp + j];
            }
            const int others = N - nbk;
            for (int j = 0; j < nbk; ++j) {
                const int p = k0 + pvt[j];
                if (p != k0 + j) {
                    double* r1 = A + (int64_t)(k0 + j) * N;
                    double* r2 = A + (int64_t)p * N;
                    for (int q = tid; q < others; q += blockDim.x) {
                        const int col = q < k0 ? q : q + nbk;
                        const double t = r1[col];
                        r1[col] = r2[col];
                        r2[col] = t;
                    }
                }
                __syncthreads();
            }
            const int c0 = k0 + nbk, nc = N - c0;
            if (nc <= 0) break;
            // (c) U12 = L11^{-1} A12: one column per thread, down the panel's rows
            for (int q = tid; q < nc; q += blockDim.x) {
                double col[kBjNbMax];
#pragma unroll
                for (int i = 0; i < kBjNbMax; ++i)
                    if (i < nbk) col[i] = A[(int64_t)(k0 + i) * N + c0 + q];
#pragma unroll
                for (int i = 1; i < kBjNbMax; ++i) {
                    if (i < nbk) {
                        double s = col[i];
#pragma unroll
                        for (int p2 = 0; p2 < kBjNbMax; ++p2)
                            if (p2 < i) s -= pan[i * pp + p2] * col[p2];
                        col[i] = s;
                    }
                }
#pragma unroll
                for (int i = 1; i < kBjNbMax; ++i)
                    if (i < nbk) A[(int64_t)(k0 + i) * N + c0 + q] = col[i];
            }
            __syncthreads();
            // (d) A22 -= L21 U12 in 16 x 16 tiles (rows c0.., columns c0..)
            const int tr = (nc + 15) / 16;
            for (int t = w; t < tr * tr; t += 4) {
                const int r0 = c0 + (t / tr) * 16, q0 = c0 + (t % tr) * 16;
                const int col = q0 + c;
                doublex4 acc;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = r0 + g + 4 * v;
                    acc[v] = (row < N && col < N) ? A[(int64_t)row * N + col] : 0.0;
                }
                const int arow = r0 + c - k0;  // panel row of this lane's A operand
                for (int p0 = 0; p0 < nbk; p0 += 4) {
                    const int kk = p0 + g;
                    const double a = (kk < nbk && r0 + c < N) ? -pan[arow * pp + kk] : 0.0;
                    const double b = (kk < nbk && col < N) ? A[(int64_t)(k0 + kk) * N + col] : 0.0;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = r0 + g + 4 * v;
                    if (row < N && col < N) A[(int64_t)row * N + col] = acc[v];
                }
            }
            __syncthreads();
        }
        if (tid == 0) status[e] = st;
        __syncthreads();
    }
}

// one workgroup per (element, rhs); x in LDS, the diagonal blocks of the
// triangles staged in LDS (64 x 65)
__global__ void __launch_bounds__(256) k_bj_solve(int64_t E, int N, int nrhs, const double* lu,
                                                  const int32_t* piv, const double* r, double* z) {
    extern __shared__ double xs[];   // [N]
    double* blk = xs + N;            // [64][65]
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    for (int64_t it = blockIdx.x; it < E * nrhs; it += gridDim.x) {
        const int64_t e = it / nrhs;
        const double* L = lu + e * (int64_t)N * N;
        const int32_t* P = piv + e * (int64_t)N;
        for (int i = tid; i < N; i += blockDim.x) xs[i] = r[it * N + i];
        __syncthreads();
        if (tid == 0)
            for (int k = 0; k < N; ++k) {
                const int p = P[k];
                if (p != k) {
                    const double t = xs[k];
                    xs[k] = xs[p];
                    xs[p] = t;
                }
            }
        __syncthreads();
        // forward: unit lower triangle
        for (int kb = 0; kb < N; kb += 64) {
            const int bs = N - kb < 64 ? N - kb : 64;
            // rows of the block minus the part left of it
            for (int i = kb + w; i < kb + bs; i += 4) {
                const double* row = L + (int64_t)i * N;
                double s = 0.0;
                for (int k = l; k < kb; k += 64) s += row[k] * xs[k];
                s = bj_wave_sum(s);
                if (l == 0) xs[i] -= s;
            }
            for (int t = tid; t < bs * bs; t += blockDim.x) {
                const int i = t / bs, k = t % bs;
                blk[i * 65 + k] = L[(int64_t)(kb + i) * N + kb + k];
            }
            __syncthreads();
            if (w == 0) {
                double xi = l < bs ? xs[kb + l] : 0.0;
                for (int k = 0; k < bs; ++k) {
                    const double xk = __shfl(xi, k, 64);
                    if (l > k && l < bs) xi -= blk[l * 65 + k] * xk;
                }
                if (l < bs) xs[kb + l] = xi;
            }
            __syncthreads();
        }
        // backward: upper triangle with its diagonal
        const int nblk = (N + 63) / 64;
        for (int bi = nblk - 1; bi >= 0; --bi) {
            const int kb = bi * 64;
            const int bs = N - kb < 64 ? N - kb : 64;
            for (int i = kb + w; i < kb + bs; i += 4) {
                const double* row = L + (int64_t)i * N;
                double s = 0.0;
                for (int k = kb + bs + l; k < N; k += 64) s += row[k] * xs[k];
                s = bj_wave_sum(s);
                if (l == 0) xs[i] -= s;
            }
            for (int t = tid; t < bs * bs; t += blockDim.x) {
                const int i = t / bs, k = t % bs;
                blk[i * 65 + k] = L[(int64_t)(kb + i) * N + kb + k];
            }
            __syncthreads();
            if (w == 0) {
                double xi = l < bs ? xs[kb + l] : 0.0;
                for (int k = bs - 1; k >= 0; --k) {
                    if (l == k) xi /= blk[l * 65 + l];
                    const double xk = __shfl(xi, k, 64);
                    if (l < k) xi -= blk[l * 65 + k] * xk;
                }
                if (l < bs) xs[kb + l] = xi;
            }
            __syncthreads();
        }
        for (int i = tid; i < N; i += blockDim.x) z[it * N + i] = xs[i];
        __syncthreads();
    }
}

hipError_t launch_bj_factor(hipStream_t s, int64_t E, int N, const double* blocks, double* lu,
                            int32_t* piv, int32_t* status) {
    const int nb = bj_panel_width(N);
    const size_t lds = (size_t)N * (nb + 1) * sizeof(double);
    int grid = (int)(E < 65536 ? E : 65536);
    hipLaunchKernelGGL(k_bj_factor, dim3(grid), dim3(256), lds, s, E, N, nb, blocks, lu, piv, status);
    return hipGetLastError();
}

hipError_t launch_bj_solve(hipStream_t s, int64_t E, int N, int nrhs, const double* lu,
                           const int32_t* piv, const double* r, double* z) {
    int64_t work = E * nrhs;
    int grid = (int)(work < 65536 ? work : 65536);
    const size_t lds = ((size_t)N + 64 * 65) * sizeof(double);
    hipLaunchKernelGGL(k_bj_solve, dim3(grid), dim3(256), lds, s, E, N, nrhs, lu, piv, r, z);
    return hipGetLastError();
}

}  // namespace kp
