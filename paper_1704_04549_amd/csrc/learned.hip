// Learned setup kernels: the per-element acceptance test of predicted factors
// (learned.h) and the mask of the cold-start fallback.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "learned.h"

namespace kp {

// One workgroup per element (persistent).  LDS: mass n^d, Xax 3 n^2, work 7 n^2.
__global__ void __launch_bounds__(256) k_learned_check(int64_t E, int dim, int n, const Tables1D* tab,
                                                       const double* params, const double* factors,
                                                       double* sigma, int32_t* status, double* guess,
                                                       int32_t* accept, double factor) {
    extern __shared__ double lds[];
    __shared__ double red[4 * kMaxReduce];
    __shared__ Tables1D T;
    __shared__ double out[8];
    BlockTeam tm{red};
    {
        const double* src = (const double*)tab;
        double* dst = (double*)&T;
        for (int i = threadIdx.x; i < (int)(sizeof(Tables1D) / sizeof(double)); i += blockDim.x)
            dst[i] = src[i];
        __syncthreads();
    }
    const int nn = n * n;
    const long nd = dim == 2 ? nn : (long)nn * n;
    const int nb = dim == 3 ? 5 : 4;
    double* mass = lds;
    double* Xax = mass + nd;
    double* work = Xax + 3 * nn;
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const double* F = factors + e * nb * nn;
        const bool ok = learned_check(tm, dim, n, T, params + e * kRecLen, F, mass, Xax, work, factor, out);
        // Lanczos starts: vec A1 (and vec B1 for the second stage in 3D)
        const int gs = dim == 3 ? 2 : 1;
        for (int t = threadIdx.x; t < gs * nn; t += blockDim.x) guess[e * gs * nn + t] = F[t];
        if (threadIdx.x == 0) {
            accept[e] = ok ? 1 : 0;
            status[e] = ok ? 0 : kStatusLearnedRejected;
            for (int j = 0; j < 4; ++j) sigma[e * 4 + j] = j < 3 ? out[3 + j] : 0.0;
        }
        __syncthreads();
    }
}

hipError_t launch_learned_check(hipStream_t s, int64_t E, int dim, int n, const Tables1D* tab,
                                const double* params, const double* factors, double* sigma,
                                int32_t* status, double* guess, int32_t* accept, double factor) {
    if (E <= 0) return hipSuccess;
    const long nn = (long)n * n;
    const long nd = dim == 2 ? nn : nn * n;
    const size_t lds = (nd + 3 * nn + 7 * nn) * sizeof(double);
    const int grid = (int)(E < 65536 ? E : 65536);
    hipLaunchKernelGGL(k_learned_check, dim3(grid), dim3(256), lds, s, E, dim, n, tab, params, factors, sigma,
                       status, guess, accept, factor);
    return hipGetLastError();
}

// warm mode: guesses only (vec A1, and vec B1 in 3D)
__global__ void k_learned_guess(int64_t E, int dim, int nn, const double* factors, double* guess,
                                int32_t* accept) {
    const int nb = dim == 3 ? 5 : 4, gs = dim == 3 ? 2 : 1;
    const long count = E * (long)gs * nn;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < count; q += (long)gridDim.x * blockDim.x) {
        const long e = q / (gs * nn), t = q % (gs * nn);
        guess[q] = factors[e * nb * nn + t];
        if (t == 0) accept[e] = 0;
    }
}

hipError_t launch_learned_guess(hipStream_t s, int64_t E, int dim, int n, const double* factors, double* guess,
                                int32_t* accept) {
    if (E <= 0) return hipSuccess;
    const long count = E * (long)(dim == 3 ? 2 : 1) * n * n;
    long g = (count + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_learned_guess, dim3((int)g), dim3(256), 0, s, E, dim, n * n, factors, guess, accept);
    return hipGetLastError();
}

__global__ void k_fallback_mask(int64_t E, const int32_t* accept, const int32_t* status, int32_t* skip) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x)
        skip[e] = (accept[e] || !(status[e] & 1)) ? 1 : 0;
}

hipError_t launch_fallback_mask(hipStream_t s, int64_t E, const int32_t* accept, const int32_t* status,
                                int32_t* skip) {
    if (E <= 0) return hipSuccess;
    int64_t g = (E + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_fallback_mask, dim3((int)g), dim3(256), 0, s, E, accept, status, skip);
    return hipGetLastError();
}

}  // namespace kp
