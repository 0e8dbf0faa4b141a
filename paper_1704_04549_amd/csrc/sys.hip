// Kernels of the systems blocks (sys.h): the KSVD runs one workgroup per
// element in a persistent grid, its Lanczos work and Gram in a per-workgroup
// slot of global workspace; the tables run one workgroup per element with
// their work matrices in LDS; the apply runs one workgroup per (element,
// right-hand side) with the element's vector in LDS.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "sys.h"

namespace kp {

__global__ void __launch_bounds__(256) k_sys_ksvd(int64_t E, int nc, int n, const double* blocks, char* pc,
                                                  SysLayout L, double* ws, int64_t ws_stride) {
    __shared__ double red[4 * kMaxReduce];
    BlockTeam tm{red};
    const int m = nc * n;
    const long bsz = (long)m * n * m * n;
    double* tw = nullptr;
    SetupWork W = carve_sys(ws + blockIdx.x * ws_stride, m, n, &tw);
    double* factors = (double*)(pc + L.factors);
    double* sigma = (double*)(pc + L.sigma);
    int32_t* status = (int32_t*)(pc + L.status);
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const int st = setup_sys_element(tm, m, n, blocks + e * bsz, factors + e * L.nf, sigma + e * 4, W);
        if (threadIdx.x == 0) status[e] = st;
        __syncthreads();
    }
}

// the pair rotation's angle of every element (sys_angle_search_grp)
__global__ void __launch_bounds__(256) k_sys_rotation(int64_t E, int nc, int n, const char* pc, SysLayout L,
                                                      int32_t* angle) {
    __shared__ double red[4 * kMaxReduce];
    BlockTeam tm{red};
    const int m = nc * n;
    const double* factors = (const double*)(pc + L.factors);
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const int k = sys_angle_search_grp(tm, m, n, factors + e * L.nf);
        if (threadIdx.x == 0) angle[e] = k;
        __syncthreads();
    }
}

// inversion data with its work matrices in LDS (sys_tables_work_doubles
// doubles of dynamic LDS), then the FP32 copy of the element's tables
__global__ void __launch_bounds__(256) k_sys_tables(int64_t E, int nc, int n, char* pc, SysLayout L,
                                                    const int32_t* angle) {
    extern __shared__ double lds[];
    __shared__ double red[4 * kMaxReduce];
    __shared__ double sh[kMaxN + 8];
    BlockTeam tm{red};
    const int m = nc * n;
    const double* factors = (const double*)(pc + L.factors);
    int32_t* status = (int32_t*)(pc + L.status);
    double* tab64 = (double*)(pc + L.tab64);
    float* tab32 = (float*)(pc + L.tab32);
    int8_t* kinds = (int8_t*)(pc + L.kinds);
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        double* tab = tab64 + e * L.ne;
        const int st = tables_sys(tm, m, n, factors + e * L.nf, tab, kinds + e * kMaxN, lds, sh, angle[e]);
        float* t32 = tab32 + e * L.ne;
        for (long t = threadIdx.x; t < L.ne; t += blockDim.x) t32[t] = (float)tab[t];
        if (threadIdx.x == 0) status[e] |= st;
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

// one workgroup per element, the (m n)^2 entries row by row (coalesced stores)
__global__ void __launch_bounds__(256) k_build_sys_blocks(int64_t E, int nc, int n, const Tables1D* tab,
                                                          const double* recs, double* out) {
    const long N = (long)nc * n * n;
    const long rl = sys_rec_len(nc);
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const double* rec = recs + e * rl;
        double* A = out + e * N * N;
        for (long t = threadIdx.x; t < N * N; t += blockDim.x) A[t] = sys_block_entry(nc, n, t / N, t % N, rec, *tab);
    }
}

// y = blockdiag(A_e) x: one workgroup per element, x in LDS, one wave per row
// (its 64 lanes read 64 consecutive entries per step), four rows at a time
__global__ void __launch_bounds__(256) k_sys_operator(int64_t E, int N, const double* blocks, const double* x,
                                                      double* y) {
    extern __shared__ double xs[];
    const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const double* xe = x + e * N;
        for (int t = threadIdx.x; t < N; t += blockDim.x) xs[t] = xe[t];
        __syncthreads();
        const double* A = blocks + e * (int64_t)N * N;
        for (int i = wv; i < N; i += 4) {
            const double* row = A + (int64_t)i * N;
            double acc = 0.0;
            for (int a = lane; a < N; a += 64) acc += row[a] * xs[a];
            acc = wave_sum(acc);
            if (lane == 0) y[e * N + i] = acc;
        }
        __syncthreads();
    }
}

hipError_t launch_build_sys_blocks(hipStream_t s, int64_t E, int nc, int n, const Tables1D* tab, const double* recs,
                                   double* out) {
    if (E <= 0) return hipSuccess;
    const int grid = (int)(E < 65536 ? E : 65536);
    hipLaunchKernelGGL(k_build_sys_blocks, dim3(grid), dim3(256), 0, s, E, nc, n, tab, recs, out);
    return hipGetLastError();
}

hipError_t launch_sys_operator(hipStream_t s, int64_t E, int N, const double* blocks, const double* x, double* y) {
    if (E <= 0) return hipSuccess;
    const int grid = (int)(E < 65536 ? E : 65536);
    hipLaunchKernelGGL(k_sys_operator, dim3(grid), dim3(256), N * sizeof(double), s, E, N, blocks, x, y);
    return hipGetLastError();
}

hipError_t launch_setup_sys(hipStream_t s, int grid, int64_t E, int nc, int n, const double* blocks,
                            char* precond, double* ws, int64_t ws_stride, int32_t* angle) {
    if (E <= 0) return hipSuccess;
    SysLayout L;
    if (!sys_layout(nc, n, E, &L)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sys_ksvd, dim3(grid), dim3(256), 0, s, E, nc, n, blocks, precond, L, ws, ws_stride);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int g2 = (int)(E < 65536 ? E : 65536);
    hipLaunchKernelGGL(k_sys_rotation, dim3(g2), dim3(256), 0, s, E, nc, n, precond, L, angle);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    const int m = nc * n;
    const size_t lds = (size_t)sys_tables_work_doubles(m, n) * sizeof(double);
    hipLaunchKernelGGL(k_sys_tables, dim3(g2), dim3(256), lds, s, E, nc, n, precond, L, angle);
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
