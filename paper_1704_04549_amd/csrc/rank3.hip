// Rank-3 2D apply kernel: one workgroup per (element, right-hand side), the
// whole inner flexible GMRES in LDS (see rank3.h); with only, the elements
// not flagged there are skipped.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "rank3.h"

namespace kp {

template <typename T, typename TT, class Rnd>
__global__ void __launch_bounds__(256) k_apply_rank3(int64_t E, int n, int nrhs, const double* factors,
                                                     const TT* tabs, int64_t tab_stride,
                                                     const int8_t* kinds, const double* r, double* z,
                                                     int m, double rtol, int maxit, Rnd rnd, const int8_t* only) {
    extern __shared__ double lds[];
    __shared__ double red[4 * kMaxReduce];
    BlockTeam tm{red};
    const int nn = n * n;
    double* work = lds;
    double* small = work + rank3_work_doubles(n, m);
    T* tw = (T*)(small + rank3_small_doubles(m));
    for (int64_t w = blockIdx.x; w < E * nrhs; w += gridDim.x) {
        const int64_t e = w / nrhs;
        if (only && !only[e]) continue;
        rank3_solve(tm, n, factors + e * 6 * nn, tabs + e * tab_stride, kinds + e * kMaxN,
                    r + w * nn, z + w * nn, work, tw, small, m, rtol, maxit, rnd);
    }
}

int rank3_restart(int n) {
    const long nn = (long)n * n;
    // (2m + 6) n^2 + 3 n^2 doubles within the budget, at most 8
    const long fit = (long)(kRank3LdsMax / sizeof(double)) / nn - 9;
    long m = fit / 2;
    if (m > 8) m = 8;
    return (int)m;
}

hipError_t launch_apply_rank3(hipStream_t s, int prec, int64_t E, int n, int nrhs,
                              const double* factors, const void* tabs, int64_t tab_stride,
                              const int8_t* kinds, const double* r, double* z, const int8_t* only) {
    const int m = rank3_restart(n);
    if (m < 2) return hipErrorInvalidValue;
    const int nn = n * n;
    const size_t lds = (rank3_work_doubles(n, m) + rank3_small_doubles(m) + 3 * nn) * sizeof(double);
    const int64_t work = E * nrhs;
    const int grid = (int)(work < 65536 ? work : 65536);
    const double rtol = rank3_rtol(prec);
    const int maxit = kRank3MaxIters;
    if (prec == 0) {
        hipLaunchKernelGGL((k_apply_rank3<double, double, RoundNone>), dim3(grid), dim3(256), lds, s, E,
                           n, nrhs, factors, (const double*)tabs, tab_stride, kinds, r, z, m, rtol,
                           maxit, RoundNone(), only);
    } else if (prec == 1) {
        hipLaunchKernelGGL((k_apply_rank3<float, float, RoundNone>), dim3(grid), dim3(256), lds, s, E,
                           n, nrhs, factors, (const float*)tabs, tab_stride, kinds, r, z, m, rtol,
                           maxit, RoundNone(), only);
    } else if (prec == 2) {
        hipLaunchKernelGGL((k_apply_rank3<float, uint16_t, RoundBf16>), dim3(grid), dim3(256), lds, s,
                           E, n, nrhs, factors, (const uint16_t*)tabs, tab_stride, kinds, r, z, m,
                           rtol, maxit, RoundBf16(), only);
    } else {
        hipLaunchKernelGGL((k_apply_rank3<float, float, RoundBf16x2>), dim3(grid), dim3(256), lds, s,
                           E, n, nrhs, factors, (const float*)tabs, tab_stride, kinds, r, z, m, rtol,
                           maxit, RoundBf16x2(), only);
    }
    return hipGetLastError();
}

}  // namespace kp
