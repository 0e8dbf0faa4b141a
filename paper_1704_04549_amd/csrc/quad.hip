// Setup kernel of general (quadrature-data) elements (quad.h): one workgroup
// per element in a persistent grid, the Lanczos work and the operators'
// scratch in a per-workgroup slot of global workspace, the (n, mu) tables
// read from global memory (every workgroup reads the same few KB).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "quad.h"

namespace kp {

__global__ void __launch_bounds__(256) k_setup_quad(int64_t E, int dim, int n, int mu, double tau,
                                                    const QuadTables* qt, const double* c, const double* a,
                                                    const double* nu, const double* g, double* factors,
                                                    double* sigma, int32_t* status, double* ws,
                                                    int64_t ws_stride) {
    __shared__ double red[4 * kMaxReduce];
    BlockTeam tm{red};
    QuadScratch qs;
    SetupWork W = carve_quad_setup(ws + blockIdx.x * ws_stride, n, &qs);
    const long md = dim == 2 ? (long)mu * mu : (long)mu * mu * mu;
    const long mf = dim == 2 ? (long)mu : (long)mu * mu;
    const long nn = (long)n * n;
    const int nf = dim == 2 ? 4 : 5;
    Term2 T2[kQuadGroups3];
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        QuadElem el{dim, n, mu, tau, c + e * md, a + e * dim * md, nu + e * md, g + e * 2 * dim * mf};
        const int st = setup_quad_element(tm, el, *qt, factors + e * nf * nn, sigma + e * 4, W, qs, T2);
        if (threadIdx.x == 0) status[e] = st;
        __syncthreads();
    }
}

hipError_t launch_setup_quad(hipStream_t s, int grid, int64_t E, int dim, int n, int mu, double tau,
                             const QuadTables* qt, const double* c, const double* a, const double* nu,
                             const double* g, double* factors, double* sigma, int32_t* status, double* ws,
                             int64_t ws_stride) {
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_setup_quad, dim3(grid), dim3(256), 0, s, E, dim, n, mu, tau, qt, c, a, nu, g, factors,
                       sigma, status, ws, ws_stride);
    return hipGetLastError();
}

}  // namespace kp
