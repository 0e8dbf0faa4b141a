// Kernels of the systems blocks (sys.h): the setup runs one workgroup per
// element in a persistent grid, its Lanczos work, Gram and table scratch in a
// per-workgroup slot of global workspace; the apply runs one workgroup per
// (element, right-hand side) with the element's vector in LDS.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "sys.h"

namespace kp {

__global__ void __launch_bounds__(256) k_setup_sys(int64_t E, int nc, int n, const double* blocks, char* pc,
                                                   SysLayout L, double* ws, int64_t ws_stride) {
    __shared__ double red[4 * kMaxReduce];
    __shared__ double sh[kMaxN + 8];
    BlockTeam tm{red};
    const int m = nc * n;
    const long bsz = (long)m * n * m * n;
    double* tw = nullptr;
    SetupWork W = carve_sys(ws + blockIdx.x * ws_stride, m, n, &tw);
    double* factors = (double*)(pc + L.factors);
    double* sigma = (double*)(pc + L.sigma);
    int32_t* status = (int32_t*)(pc + L.status);
    double* tab64 = (double*)(pc + L.tab64);
    float* tab32 = (float*)(pc + L.tab32);
    int8_t* kinds = (int8_t*)(pc + L.kinds);
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        double* F = factors + e * L.nf;
        double* tab = tab64 + e * L.ne;
        int st = setup_sys_element(tm, m, n, blocks + e * bsz, F, sigma + e * 4, W);
        st |= tables_sys(tm, m, n, F, tab, kinds + e * kMaxN, tw, sh);
        float* t32 = tab32 + e * L.ne;
        for (long t = threadIdx.x; t < L.ne; t += blockDim.x) t32[t] = (float)tab[t];
        if (threadIdx.x == 0) status[e] = st;
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_apply_sys(int64_t E, int nc, int n, int nrhs, const T* tabs,
                                                   const int8_t* kinds, int64_t ne, const double* r, double* z) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ double red[4 * kMaxReduce];
    BlockTeam tm{red};
    T* X = (T*)lds_raw;
    const int m = nc * n;
    const int md = m * n;
    T* Y = X + md;
    T* H = Y + md;
    const int64_t item = blockIdx.x;  // e * nrhs + rhs
    const int64_t e = item / nrhs;
    const double* rv = r + item * md;
    for (int t = threadIdx.x; t < md; t += blockDim.x) X[t] = (T)rv[t];
    __syncthreads();
    apply_sys(tm, m, n, tabs + e * ne, kinds + e * kMaxN, X, Y, H);
    double* zv = z + item * md;
    for (int t = threadIdx.x; t < md; t += blockDim.x) zv[t] = (double)X[t];
}

hipError_t launch_setup_sys(hipStream_t s, int grid, int64_t E, int nc, int n, const double* blocks,
                            char* precond, double* ws, int64_t ws_stride) {
    if (E <= 0) return hipSuccess;
    SysLayout L;
    if (!sys_layout(nc, n, E, &L)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_setup_sys, dim3(grid), dim3(256), 0, s, E, nc, n, blocks, precond, L, ws, ws_stride);
    return hipGetLastError();
}

hipError_t launch_apply_sys(hipStream_t s, int64_t E, int nc, int n, int prec, int nrhs, const char* precond,
                            const double* r, double* z) {
    if (E <= 0 || nrhs <= 0) return hipSuccess;
    SysLayout L;
    if (!sys_layout(nc, n, E, &L)) return hipErrorInvalidValue;
    const int m = nc * n;
    const int64_t items = E * nrhs;
    if (items > 0x7fffffff) return hipErrorInvalidValue;
    const int8_t* kinds = (const int8_t*)(precond + L.kinds);
    if (prec == 0) {
        const size_t lds = (2 * (size_t)m * n + 2 * m) * sizeof(double);
        hipLaunchKernelGGL(k_apply_sys<double>, dim3((unsigned)items), dim3(256), lds, s, E, nc, n, nrhs,
                           (const double*)(precond + L.tab64), kinds, L.ne, r, z);
    } else {
        const size_t lds = (2 * (size_t)m * n + 2 * m) * sizeof(float);
        hipLaunchKernelGGL(k_apply_sys<float>, dim3((unsigned)items), dim3(256), lds, s, E, nc, n, nrhs,
                           (const float*)(precond + L.tab32), kinds, L.ne, r, z);
    }
    return hipGetLastError();
}

}  // namespace kp
