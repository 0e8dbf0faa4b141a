// HIP kernels of the KSVD preconditioner for gfx950.
//
// Setup kernels run one element per workgroup with the team routines of
// elem_ops.h; the hot apply kernels for n = 16 live in apply_mfma.hip.
#include <hip/hip_runtime.h>

#include "elem_ops.h"
#include "kernels.h"

namespace kp {

// ---------------------------------------------------------------- blocks
// One workgroup per element: structure in LDS, then every entry of the
// n^d x n^d block, row by row (coalesced stores).
__global__ void __launch_bounds__(256) k_build_blocks(int64_t E, int dim, int n, const Tables1D* tab,
                                                      const double* params, double* out) {
    extern __shared__ double lds[];
    __shared__ double red[8 * kMaxReduce];
    BlockTeam tm{red};
    const long nd = dim == 2 ? n * n : n * n * n;
    double* mass = lds;
    double* Xax = lds + nd;
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        record_structure(tm, params + e * kRecLen, *tab, dim, mass, Xax);
        double* A = out + e * nd * nd;
        for (long t = threadIdx.x; t < nd * nd; t += blockDim.x)
            A[t] = block_entry(dim, n, t / nd, t % nd, mass, Xax, tab->w);
        __syncthreads();
    }
}

// ----------------------------------------------------------------- setup
// Persistent grid: workgroup g handles elements g, g + G, ... with its own
// workspace slot.  Team = whole workgroup (256 threads).
template <bool kRefine>
__global__ void __launch_bounds__(256) k_setup(int64_t E, int dim, int n, int rank,
                                               const Tables1D* tab, const double* params,
                                               const double* blocks, const double* guess,
                                               double* factors, double* sigma, int32_t* status,
                                               double* ws, int64_t ws_stride, const int32_t* skip,
                                               int32_t status_or) {
    __shared__ double red[4 * kMaxReduce];
    __shared__ Tables1D T;
    extern __shared__ double small[];
    BlockTeam tm{red};
    // copy the tables once into LDS
    {
        const double* src = (const double*)tab;
        double* dst = (double*)&T;
        for (int i = threadIdx.x; i < (int)(sizeof(Tables1D) / sizeof(double)); i += blockDim.x)
            dst[i] = src[i];
        __syncthreads();
    }
    const bool expl = blocks != nullptr;
    SetupWork W = carve_setup_work(ws + blockIdx.x * ws_stride, dim, n, expl, rank);
    carve_small(small, n, expl, &W);
    const long nn = (long)n * n;
    const long nd = dim == 2 ? nn : nn * n;
    const int nf = dim == 2 ? 2 * rank : 5;
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        if (skip && skip[e]) continue;  // uniform across the workgroup
        const double* blk = expl ? blocks + e * nd * nd : nullptr;
        // guesses: [E][gs][n^2], gs = 2 in 3D (stage-1 and stage-2 starts), 1 in 2D
        const long gs = dim == 3 ? 2 : 1;
        const double* g = guess ? guess + e * gs * nn : nullptr;
        const double* g2 = (guess && dim == 3) ? g + nn : nullptr;
        int st = setup_element<kRefine>(tm, dim, n, rank, T, params + e * kRecLen, blk, g,
                               factors + e * nf * nn, sigma + e * 4, W, g2);
        if (threadIdx.x == 0) status[e] = st | status_or;
        __syncthreads();
    }
}

// ---------------------------------------------------------- apply tables
// Three kernels: prepare (one wave per element: pair rotation, inverses, C1
// and C2), Schur (one wave per (element, C matrix), with a small LDS
// footprint so that many run per CU) and finish (one wave per element: L
// tables, kinds, N_j).  Intermediates live in the element's own table slots.
__global__ void __launch_bounds__(64) k_tables_prepare(int64_t E, int dim, int n, int rank,
                                                       const double* factors, double* tab64,
                                                       int32_t* status) {
    extern __shared__ double lds[];
    __shared__ double red[kMaxReduce];
    __shared__ double sh[kMaxN + 8];
    __shared__ int ipiv[kMaxN];
    BlockTeam tm{red};
    const long nn = (long)n * n;
    const int nf = dim == 2 ? 2 * rank : 5;
    const long ne = tab_entries(n);
    double* F = lds;              // nf n^2
    double* work = F + nf * nn;   // 10 n^2
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        for (long t = threadIdx.x; t < nf * nn; t += blockDim.x) F[t] = factors[e * nf * nn + t];
        __syncthreads();
        double* tab = tab64 + e * ne;
        const int st = tables_prepare(tm, dim, n, rank, F, tab, tab + 7 * nn, work, ipiv, sh);
        if (threadIdx.x == 0) status[e] |= st;
        __syncthreads();
    }
}

// work item w = 2 e + i: real Schur form of C_(i+1), held in N slot i, into
// the T_(i+1) and R_i slots
__global__ void __launch_bounds__(64) k_tables_schur(int64_t E, int n, double* tab64,
                                                     int32_t* status) {
    extern __shared__ double lds[];
    __shared__ double red[kMaxReduce];
    __shared__ double sh[kMaxN + 8];
    BlockTeam tm{red};
    const long nn = (long)n * n;
    const long ne = tab_entries(n);
    double* H = lds;
    double* Q = lds + nn;
    for (int64_t w = blockIdx.x; w < 2 * E; w += gridDim.x) {
        const int64_t e = w >> 1;
        const int i = (int)(w & 1);
        double* tab = tab64 + e * ne;
        const int st = tables_schur(tm, n, tab + (7 + i) * nn, tab + (5 + i) * nn,
                                    tab + (3 + i) * nn, H, Q, sh);
        if (threadIdx.x == 0 && st) atomicOr(&status[e], st);
        __syncthreads();
    }
}

__global__ void __launch_bounds__(64) k_tables_finish(int64_t E, int dim, int n, double* tab64,
                                                      int8_t* kinds, int32_t* status) {
    extern __shared__ double lds[];  // 6 n^2 work doubles
    __shared__ double red[kMaxReduce];
    __shared__ double sh[kMaxN + 8];
    __shared__ int ipiv[kMaxN];
    BlockTeam tm{red};
    const long nn = (long)n * n;
    const long ne = tab_entries(n);
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        double* tab = tab64 + e * ne;
        const int st = tables_finish(tm, dim, n, tab, tab + 7 * nn, kinds + e * kMaxN, lds, ipiv, sh);
        if (threadIdx.x == 0) status[e] |= st;
        __syncthreads();
    }
}

// FP32 and split-BF16 copies of the FP64 tables: hi = bf16(f), lo = bf16(f - hi),
// and their sum hi + lo as a float (the value the split operands carry)
__global__ void k_cast_tables(int64_t count, const double* t64, float* t32, uint16_t* hi,
                              uint16_t* lo, float* t2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = t64[i];
        const float f = (float)v;
        t32[i] = f;
        const uint16_t h = f32_to_bf16(f);
        const uint16_t l = f32_to_bf16(f - bf16_to_f32(h));
        hi[i] = h;
        lo[i] = l;
        t2[i] = bf16_to_f32(h) + bf16_to_f32(l);
    }
}

// --------------------------------------------------------- generic apply
// One workgroup per (element, rhs); tensor in LDS, tables read from global.
template <typename T, typename TT, class Rnd>
__global__ void __launch_bounds__(256) k_apply_generic(int64_t E, int dim, int n, int nrhs,
                                                       const TT* tabs, int64_t tab_stride,
                                                       const int8_t* kinds, const double* r,
                                                       double* z, Rnd rnd) {
    extern __shared__ double lds[];
    __shared__ double red[4 * kMaxReduce];
    BlockTeam tm{red};
    const long nd = dim == 2 ? n * n : n * n * n;
    T* X = (T*)lds;
    T* Y = X + nd;
    T* H = Y + nd;
    for (int64_t w = blockIdx.x; w < E * nrhs; w += gridDim.x) {
        const int64_t e = w / nrhs;
        for (long t = threadIdx.x; t < nd; t += blockDim.x) X[t] = (T)r[w * nd + t];
        __syncthreads();
        apply_tensor(tm, dim, n, tabs + e * tab_stride, kinds + e * kMaxN, X, Y, H, rnd);
        for (long t = threadIdx.x; t < nd; t += blockDim.x) z[w * nd + t] = (double)X[t];
        __syncthreads();
    }
}

// ------------------------------------------------- host-side launchers
hipError_t launch_build_blocks(hipStream_t s, int64_t E, int dim, int n, const Tables1D* tab,
                               const double* params, double* out) {
    const long nd = dim == 2 ? n * n : n * n * n;
    size_t lds = (nd + 3 * n * n) * sizeof(double);
    int grid = (int)(E < 65536 ? E : 65536);
    hipLaunchKernelGGL(k_build_blocks, dim3(grid), dim3(256), lds, s, E, dim, n, tab, params, out);
    return hipGetLastError();
}

hipError_t launch_setup(hipStream_t s, int grid, int64_t E, int dim, int n, int rank,
                        const Tables1D* tab, const double* params, const double* blocks,
                        const double* guess, double* factors, double* sigma, int32_t* status,
                        double* ws, int64_t ws_stride, const int32_t* skip, int32_t status_or) {
    const size_t lds = setup_small_doubles(n, blocks != nullptr) * sizeof(double);
    auto kern = rank >= 3 ? k_setup<true> : k_setup<false>;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, s, E, dim, n, rank, tab, params, blocks,
                       guess, factors, sigma, status, ws, ws_stride, skip, status_or);
    return hipGetLastError();
}

hipError_t launch_form_tables(hipStream_t s, int64_t E, int dim, int n, int rank,
                              const double* factors, double* tab64, int8_t* kinds,
                              int32_t* status) {
    if (E <= 0) return hipSuccess;
    const long nn = (long)n * n;
    const int nf = dim == 2 ? 2 * rank : 5;
    // at most (6 + 10) 32^2 doubles = 128 KiB of LDS (2D rank 3, n = 32)
    const size_t lds = (nf + 10) * nn * sizeof(double);
    const int grid = (int)(E < 65536 ? E : 65536);
    hipLaunchKernelGGL(k_tables_prepare, dim3(grid), dim3(64), lds, s, E, dim, n, rank, factors,
                       tab64, status);
    const int64_t items = 2 * E;
    const int grid2 = (int)(items < 65536 ? items : 65536);
    hipLaunchKernelGGL(k_tables_schur, dim3(grid2), dim3(64), 2 * nn * sizeof(double), s, E, n,
                       tab64, status);
    hipLaunchKernelGGL(k_tables_finish, dim3(grid), dim3(64), 6 * nn * sizeof(double), s, E, dim, n,
                       tab64, kinds, status);
    return hipGetLastError();
}

// fragment-ordered copies of the n = 16 tables for the matrix-core apply:
// one thread per (element, matrix, lane)
__global__ void k_frag_tables(int64_t E, const double* t64, double* f64f, float* f32f, uint16_t* fbf,
                              uint16_t* fbf3) {
    const int64_t count = E * 23 * 64;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < count;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(q % 64);
        const int64_t em = q / 64;  // element * 23 + matrix
        const int g = l >> 4, c = l & 15;
        const double* M = t64 + em * 256;
        for (int k = 0; k < 4; ++k) {
            const double v = M[c * 16 + 4 * k + g];
            f64f[q * 4 + k] = v;
            f32f[q * 4 + k] = (float)v;
        }
        const int64_t e = em / 23, m = em % 23;
        for (int i = 0; i < 4; ++i) {
            const float f = (float)M[c * 16 + 4 * g + i];
            const uint16_t h = f32_to_bf16(f);
            fbf[q * 4 + i] = h;
            fbf3[((e * 23 + m) * 2 + 0) * 256 + l * 4 + i] = h;
            fbf3[((e * 23 + m) * 2 + 1) * 256 + l * 4 + i] = f32_to_bf16(f - bf16_to_f32(h));
        }
    }
}

hipError_t launch_frag_tables(hipStream_t s, int64_t E, const double* t64, double* f64f, float* f32f,
                              uint16_t* fbf, uint16_t* fbf3) {
    const int64_t count = E * 23 * 64;
    int grid = (int)((count + 255) / 256);
    if (grid > 65536) grid = 65536;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_frag_tables, dim3(grid), dim3(256), 0, s, E, t64, f64f, f32f, fbf, fbf3);
    return hipGetLastError();
}

hipError_t launch_cast_tables(hipStream_t s, int64_t count, const double* t64, float* t32,
                              uint16_t* hi, uint16_t* lo, float* t2) {
    int grid = (int)((count + 255) / 256);
    if (grid > 65536) grid = 65536;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_cast_tables, dim3(grid), dim3(256), 0, s, count, t64, t32, hi, lo, t2);
    return hipGetLastError();
}

hipError_t launch_apply_generic(hipStream_t s, int prec, int64_t E, int dim, int n, int nrhs,
                                const void* tabs, int64_t tab_stride, const int8_t* kinds,
                                const double* r, double* z) {
    const long nd = dim == 2 ? n * n : n * n * n;
    int64_t work = E * nrhs;
    int grid = (int)(work < 65536 ? work : 65536);
    if (prec == 0) {
        size_t lds = 4 * nd * sizeof(double);
        hipLaunchKernelGGL((k_apply_generic<double, double, RoundNone>), dim3(grid), dim3(256), lds, s,
                           E, dim, n, nrhs, (const double*)tabs, tab_stride, kinds, r, z, RoundNone());
    } else if (prec == 1) {
        size_t lds = 4 * nd * sizeof(float);
        hipLaunchKernelGGL((k_apply_generic<float, float, RoundNone>), dim3(grid), dim3(256), lds, s,
                           E, dim, n, nrhs, (const float*)tabs, tab_stride, kinds, r, z, RoundNone());
    } else if (prec == 2) {
        size_t lds = 4 * nd * sizeof(float);
        hipLaunchKernelGGL((k_apply_generic<float, uint16_t, RoundBf16>), dim3(grid), dim3(256), lds,
                           s, E, dim, n, nrhs, (const uint16_t*)tabs, tab_stride, kinds, r, z,
                           RoundBf16());
    } else {
        size_t lds = 4 * nd * sizeof(float);
        hipLaunchKernelGGL((k_apply_generic<float, float, RoundBf16x2>), dim3(grid), dim3(256), lds,
                           s, E, dim, n, nrhs, (const float*)tabs, tab_stride, kinds, r, z,
                           RoundBf16x2());
    }
    return hipGetLastError();
}

}  // namespace kp
