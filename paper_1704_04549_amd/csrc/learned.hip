// Learned setup kernels: the per-element judge of predicted factors against
// the SVD's (learned.h), the Lanczos starts and the mask of the cold-start
// fallback.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "learned.h"

namespace kp {

// One workgroup per element (persistent).  LDS: judge_work_doubles.
// pred: predicted factors [E][nf][n][n]; factors: the SVD's factors with
// their FP64 apply tables tab64 [E][tab_stride] and kinds [E][kMaxN].
// out [E][4] (res_p, res_s, ||A||, gamma) and accept [E] may be NULL.  With
// use_pred set, an accepted element's prediction replaces its factors and its
// status becomes 0; a rejected element's status gains status_rejected.
__global__ void __launch_bounds__(256) k_learned_judge(int64_t E, int dim, int n, const Tables1D* tab,
                                                       const double* params, const double* pred,
                                                       double* factors, const double* tab64, int64_t tab_stride,
                                                       const int8_t* kinds, double factor, double guard,
                                                       double* out, int32_t* accept, int32_t* status,
                                                       int use_pred, int32_t status_rejected) {
    extern __shared__ double lds[];
    __shared__ double red[4 * kMaxReduce];
    __shared__ double res[4];
    BlockTeam tm{red};
    const long nn = (long)n * n;
    const int nb = dim == 3 ? 5 : 4;
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const double* Fp = pred + e * nb * nn;
        double* Fs = factors + e * nb * nn;
        const bool ok = learned_judge(tm, dim, n, *tab, params + e * kRecLen, Fp, Fs, tab64 + e * tab_stride,
                                      kinds + e * kMaxN, lds, factor, guard, res);
        if (use_pred && ok)
            for (long t = threadIdx.x; t < nb * nn; t += blockDim.x) Fs[t] = Fp[t];
        if (threadIdx.x == 0) {
            if (out)
                for (int j = 0; j < 4; ++j) out[e * 4 + j] = res[j];
            if (accept) accept[e] = ok ? 1 : 0;
            if (use_pred && status) status[e] = ok ? 0 : (status[e] | status_rejected);
        }
        __syncthreads();
    }
}

size_t learned_judge_lds(int dim, int n) { return (size_t)judge_work_doubles(dim, n) * sizeof(double); }

hipError_t launch_learned_judge(hipStream_t s, int64_t E, int dim, int n, const Tables1D* tab,
                                const double* params, const double* pred, double* factors, const double* tab64,
                                int64_t tab_stride, const int8_t* kinds, double factor, double guard,
                                double* out, int32_t* accept, int32_t* status, bool use_pred,
                                int32_t status_rejected) {
    if (E <= 0) return hipSuccess;
    const size_t lds = learned_judge_lds(dim, n);
    const int grid = (int)(E < 65536 ? E : 65536);
    hipLaunchKernelGGL(k_learned_judge, dim3(grid), dim3(256), lds, s, E, dim, n, tab, params, pred, factors,
                       tab64, tab_stride, kinds, factor, guard, out, accept, status, use_pred ? 1 : 0,
                       status_rejected);
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
