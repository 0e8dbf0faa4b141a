// Exact block Jacobi: batched LU with partial pivoting of the explicit
// diagonal blocks and the matching triangular solves.  The comparator of the
// paper (Sec. 5): O(N^3) form and O(N^2) apply per element, N = n^d.
//
// LU factors are stored column-major per element (lu[e][j*N + i] = entry (i, j)),
// unit lower triangle below the diagonal, U on and above it; piv[e][k] is the
// row swapped with row k at step k.
#include <hip/hip_runtime.h>

#include "kp_common.h"
#include "krylov.h"

namespace kp {

__global__ void __launch_bounds__(256) k_bj_factor(int64_t E, int N, const double* blocks,
                                                   double* lu, int32_t* piv, int32_t* status) {
    __shared__ double vmax[4];
    __shared__ int imax[4];
    __shared__ int pk;
    const int nw = blockDim.x >> 6, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const double* A = blocks + e * (int64_t)N * N;
        double* L = lu + e * (int64_t)N * N;
        int32_t* P = piv + e * (int64_t)N;
        // transpose copy: row-major block -> column-major factors
        for (int64_t t = threadIdx.x; t < (int64_t)N * N; t += blockDim.x) {
            const int i = (int)(t / N), j = (int)(t % N);
            L[(int64_t)j * N + i] = A[t];
        }
        int st = 0;
        __syncthreads();
        for (int k = 0; k < N; ++k) {
            double* colk = L + (int64_t)k * N;
            // pivot: largest |entry| of column k at or below the diagonal (lowest index on ties)
            double bv = -1.0;
            int bi = k;
            for (int i = k + threadIdx.x; i < N; i += blockDim.x) {
                const double v = fabs(colk[i]);
                if (v > bv) { bv = v; bi = i; }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(bv, off, 64);
                const int oi = __shfl_xor(bi, off, 64);
                if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
            }
            if (lane == 0) { vmax[wv] = bv; imax[wv] = bi; }
            __syncthreads();
            if (threadIdx.x == 0) {
                double b = vmax[0];
                int ii = imax[0];
                for (int q = 1; q < nw; ++q)
                    if (vmax[q] > b || (vmax[q] == b && imax[q] < ii)) { b = vmax[q]; ii = imax[q]; }
                pk = ii;
                P[k] = ii;
            }
            __syncthreads();
            const int p = pk;
            if (p != k)
                for (int j = threadIdx.x; j < N; j += blockDim.x) {
                    double* cj = L + (int64_t)j * N;
                    const double t = cj[k];
                    cj[k] = cj[p];
                    cj[p] = t;
                }
            __syncthreads();
            const double pv = colk[k];
            if (pv == 0.0) {
                st |= 2;
                continue;
            }
            for (int i = k + 1 + threadIdx.x; i < N; i += blockDim.x) colk[i] /= pv;
            __syncthreads();
            const int m = N - k - 1;
            for (int64_t t = threadIdx.x; t < (int64_t)m * m; t += blockDim.x) {
                const int j = k + 1 + (int)(t / m), i = k + 1 + (int)(t % m);
                double* cj = L + (int64_t)j * N;
                cj[i] -= colk[i] * cj[k];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) status[e] = st;
        __syncthreads();
    }
}

// one workgroup per (element, rhs); the right-hand side is held in LDS
__global__ void __launch_bounds__(256) k_bj_solve(int64_t E, int N, int nrhs, const double* lu,
                                                  const int32_t* piv, const double* r, double* z) {
    extern __shared__ double xs[];
    for (int64_t w = blockIdx.x; w < E * nrhs; w += gridDim.x) {
        const int64_t e = w / nrhs;
        const double* L = lu + e * (int64_t)N * N;
        const int32_t* P = piv + e * (int64_t)N;
        for (int i = threadIdx.x; i < N; i += blockDim.x) xs[i] = r[w * N + i];
        __syncthreads();
        if (threadIdx.x == 0)
            for (int k = 0; k < N; ++k) {
                const int p = P[k];
                if (p != k) { const double t = xs[k]; xs[k] = xs[p]; xs[p] = t; }
            }
        __syncthreads();
        for (int k = 0; k < N; ++k) {  // unit lower triangle
            const double xk = xs[k];
            const double* ck = L + (int64_t)k * N;
            for (int i = k + 1 + threadIdx.x; i < N; i += blockDim.x) xs[i] -= ck[i] * xk;
            __syncthreads();
        }
        for (int k = N - 1; k >= 0; --k) {  // upper triangle
            const double* ck = L + (int64_t)k * N;
            const double xk = xs[k] / ck[k];
            __syncthreads();
            if (threadIdx.x == 0) xs[k] = xk;
            for (int i = threadIdx.x; i < k; i += blockDim.x) xs[i] -= ck[i] * xk;
            __syncthreads();
        }
        for (int i = threadIdx.x; i < N; i += blockDim.x) z[w * N + i] = xs[i];
        __syncthreads();
    }
}

hipError_t launch_bj_factor(hipStream_t s, int64_t E, int N, const double* blocks, double* lu,
                            int32_t* piv, int32_t* status) {
    int grid = (int)(E < 65536 ? E : 65536);
    hipLaunchKernelGGL(k_bj_factor, dim3(grid), dim3(256), 0, s, E, N, blocks, lu, piv, status);
    return hipGetLastError();
}

hipError_t launch_bj_solve(hipStream_t s, int64_t E, int N, int nrhs, const double* lu,
                           const int32_t* piv, const double* r, double* z) {
    int64_t work = E * nrhs;
    int grid = (int)(work < 65536 ? work : 65536);
    hipLaunchKernelGGL(k_bj_solve, dim3(grid), dim3(256), N * sizeof(double), s, E, N, nrhs, lu, piv,
                       r, z);
    return hipGetLastError();
}

}  // namespace kp
