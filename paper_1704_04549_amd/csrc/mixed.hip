// Persistent kernels over mixed batches (descriptors in mixed.h).  The
// per-element arithmetic is the same as for uniform batches (elem_ops.h);
// only the shape and the offsets come from each element's descriptor.
#include <hip/hip_runtime.h>

#include "mixed.h"

namespace kp {

// ---------------------------------------------------------------- setup
// Elements in `order` (longest first); the 1D tables of the current n are
// copied into LDS when n changes.
__global__ void __launch_bounds__(256) k_mixed_setup(int64_t E, const MixedElem* el, const int32_t* order,
                                                     Tables1D* const* tabs, const double* params,
                                                     double* factors, double* sigma, int32_t* status,
                                                     double* ws, int64_t ws_stride) {
    __shared__ double red[4 * kMaxReduce];
    __shared__ Tables1D T;
    extern __shared__ double small[];
    BlockTeam tm{red};
    int cur_n = -1;
    for (int64_t q = blockIdx.x; q < E; q += gridDim.x) {
        const int64_t e = order[q];
        const MixedElem d = el[e];
        if (d.n != cur_n) {
            __syncthreads();
            const double* src = (const double*)tabs[d.n];
            double* dst = (double*)&T;
            for (int i = threadIdx.x; i < (int)(sizeof(Tables1D) / sizeof(double)); i += blockDim.x)
                dst[i] = src[i];
            __syncthreads();
            cur_n = d.n;
        }
        SetupWork W = carve_setup_work(ws + blockIdx.x * ws_stride, d.dim, d.n, false, 2);
        carve_small(small, d.n, false, &W);
        const int st = setup_element<false>(tm, d.dim, d.n, 2, T, params + e * kRecLen, nullptr, nullptr,
                                            factors + d.fac_off, sigma + e * 4, W);
        if (threadIdx.x == 0) status[e] = st;
        __syncthreads();
    }
}

hipError_t launch_mixed_setup(hipStream_t s, int grid, int64_t E, const MixedElem* el, const int32_t* order,
                              Tables1D* const* tabs, const double* params, double* factors, double* sigma,
                              int32_t* status, double* ws, int64_t ws_stride, size_t small_doubles) {
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mixed_setup, dim3(grid), dim3(256), small_doubles * sizeof(double), s, E, el, order,
                       tabs, params, factors, sigma, status, ws, ws_stride);
    return hipGetLastError();
}

// One wave per element (four per workgroup, each with its own LDS part and
// workspace slot), for the classes whose LDS part fits four times; the 1D
// tables are read through the element's own table pointer (a workgroup can
// hold elements of different n).
__global__ void __launch_bounds__(256) k_mixed_setup_waves(int64_t E, const MixedElem* el, const int32_t* order,
                                                           Tables1D* const* tabs, const double* params,
                                                           double* factors, double* sigma, int32_t* status,
                                                           double* ws, int64_t ws_stride, int64_t small_stride) {
    extern __shared__ double small[];
    WaveTeam tm;
    const int wv = (int)(threadIdx.x >> 6);
    const int64_t slot = (int64_t)blockIdx.x * 4 + wv;
    for (int64_t q = slot; q < E; q += (int64_t)gridDim.x * 4) {
        const int64_t e = order[q];
        const MixedElem d = el[e];
        const Tables1D& T = *tabs[d.n];
        SetupWork W = carve_setup_work(ws + slot * ws_stride, d.dim, d.n, false, 2);
        carve_small(small + wv * small_stride, d.n, false, &W);
        const int st = setup_element<false>(tm, d.dim, d.n, 2, T, params + e * kRecLen, nullptr, nullptr,
                                            factors + d.fac_off, sigma + e * 4, W);
        if ((threadIdx.x & 63) == 0) status[e] = st;
        tm.sync();
    }
}

hipError_t launch_mixed_setup_waves(hipStream_t s, int grid4, int64_t E, const MixedElem* el,
                                    const int32_t* order, Tables1D* const* tabs, const double* params,
                                    double* factors, double* sigma, int32_t* status, double* ws,
                                    int64_t ws_stride, int64_t small_stride) {
    if (E <= 0) return hipSuccess;
    if (4 * small_stride * sizeof(double) > kSetupWavesLdsMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mixed_setup_waves, dim3(grid4), dim3(256), 4 * small_stride * sizeof(double), s, E, el,
                       order, tabs, params, factors, sigma, status, ws, ws_stride, small_stride);
    return hipGetLastError();
}

// ---------------------------------------------------------------- apply
// 256 threads.  Block items: the workgroup applies one element with the
// tensor, a scratch tensor (block_nd values each) and the sweep's block buffer
// in LDS.  Wave items: each wave applies its own element in its own part of
// LDS (2 wave_nd + wave_h values).
template <typename T, typename TT, class Rnd>
__global__ void __launch_bounds__(256) k_mixed_apply(int n_items, int n_block, const int32_t* items,
                                                     const MixedElem* el, const TT* tabs, const int8_t* kinds,
                                                     const double* r, double* z, long block_nd, long wave_nd,
                                                     long wave_h, Rnd rnd) {
    extern __shared__ double lds[];
    __shared__ double red[4 * kMaxReduce];
    T* base = (T*)lds;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        if (it < n_block) {
            BlockTeam tm{red};
            const int64_t e = items[(long)it * kMixedItemWidth];
            const MixedElem d = el[e];
            const long nd = d.dim == 2 ? (long)d.n * d.n : (long)d.n * d.n * d.n;
            T* X = base;
            T* Y = X + block_nd;
            T* H = Y + block_nd;
            for (long t = threadIdx.x; t < nd; t += blockDim.x) X[t] = (T)r[d.vec_off + t];
            __syncthreads();
            apply_tensor(tm, d.dim, d.n, tabs + d.tab_off, kinds + e * kMaxN, X, Y, H, rnd);
            for (long t = threadIdx.x; t < nd; t += blockDim.x) z[d.vec_off + t] = (double)X[t];
            __syncthreads();
        } else {
            WaveTeam tm;
            const int wv = threadIdx.x >> 6;
            const int64_t e = items[(long)it * kMixedItemWidth + wv];
            if (e >= 0) {
                const MixedElem d = el[e];
                const long nd = d.dim == 2 ? (long)d.n * d.n : (long)d.n * d.n * d.n;
                T* X = base + (2 * wave_nd + wave_h) * wv;
                T* Y = X + wave_nd;
                T* H = Y + wave_nd;
                for (long t = tm.tid(); t < nd; t += 64) X[t] = (T)r[d.vec_off + t];
                tm.sync();
                apply_tensor(tm, d.dim, d.n, tabs + d.tab_off, kinds + e * kMaxN, X, Y, H, rnd);
                for (long t = tm.tid(); t < nd; t += 64) z[d.vec_off + t] = (double)X[t];
                tm.sync();
            }
            // every wave finishes its element before the workgroup moves on,
            // so the next block item may reuse the whole LDS
            __syncthreads();
        }
    }
}

hipError_t launch_mixed_apply(hipStream_t s, int prec, int grid, int n_items, int n_block, const int32_t* items,
                              const MixedElem* el, const void* tabs, const int8_t* kinds, const double* r,
                              double* z, long block_nd, long block_h, long wave_nd, long wave_h) {
    if (n_items <= 0) return hipSuccess;
    const size_t lds =
        mixed_apply_lds(prec == 0 ? sizeof(double) : sizeof(float), block_nd, block_h, wave_nd, wave_h);
    if (lds > kMixedApplyLdsMax) return hipErrorInvalidValue;
    if (prec == 0)
        hipLaunchKernelGGL((k_mixed_apply<double, double, RoundNone>), dim3(grid), dim3(256), lds, s, n_items,
                           n_block, items, el, (const double*)tabs, kinds, r, z, block_nd, wave_nd, wave_h, RoundNone());
    else if (prec == 1)
        hipLaunchKernelGGL((k_mixed_apply<float, float, RoundNone>), dim3(grid), dim3(256), lds, s, n_items,
                           n_block, items, el, (const float*)tabs, kinds, r, z, block_nd, wave_nd, wave_h, RoundNone());
    else if (prec == 2)
        hipLaunchKernelGGL((k_mixed_apply<float, uint16_t, RoundBf16>), dim3(grid), dim3(256), lds, s, n_items,
                           n_block, items, el, (const uint16_t*)tabs, kinds, r, z, block_nd, wave_nd, wave_h,
                           RoundBf16());
    else
        hipLaunchKernelGGL((k_mixed_apply<float, float, RoundBf16x2>), dim3(grid), dim3(256), lds, s, n_items,
                           n_block, items, el, (const float*)tabs, kinds, r, z, block_nd, wave_nd, wave_h,
                           RoundBf16x2());
    return hipGetLastError();
}

// ------------------------------------------------------------- operator
// y = blockdiag(A_e) x for the records' structured blocks (the mixed batch is
// block-diagonal: no face coupling).  One workgroup per element.
__global__ void __launch_bounds__(256) k_mixed_operator(int64_t E, const MixedElem* el, Tables1D* const* tabs,
                                                        const double* params, const double* x, double* y) {
    extern __shared__ double lds[];
    __shared__ double red[4 * kMaxReduce];
    BlockTeam tm{red};
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const MixedElem d = el[e];
        const Tables1D& T = *tabs[d.n];
        const int n = d.n, nn = n * n;
        const long nd = d.dim == 2 ? nn : (long)nn * n;
        double* mass = lds;
        double* Xax = mass + nd;
        record_structure(tm, params + e * kRecLen, T, d.dim, mass, Xax);  // ends with a barrier
        const double* xe = x + d.vec_off;
        for (long I = threadIdx.x; I < nd; I += blockDim.x) {
            double v = mass[I] * xe[I];
            int idx[3];
            if (d.dim == 2) { idx[0] = (int)(I / n); idx[1] = (int)(I % n); }
            else { idx[0] = (int)(I / nn); idx[1] = (int)((I / n) % n); idx[2] = (int)(I % n); }
            for (int ax = 0; ax < d.dim; ++ax) {
                long stride = 1;
                for (int k = ax + 1; k < d.dim; ++k) stride *= n;
                double wp = 1.0;
                for (int k = 0; k < d.dim; ++k)
                    if (k != ax) wp *= T.w[idx[k]];
                const double* Xr = Xax + ax * nn + idx[ax] * n;
                const long b0 = I - idx[ax] * stride;
                double sacc = 0.0;
                #pragma unroll 8
                for (int k = 0; k < n; ++k) sacc += Xr[k] * xe[b0 + k * stride];
                v += wp * sacc;
            }
            y[d.vec_off + I] = v;
        }
        __syncthreads();
    }
}

hipError_t launch_mixed_operator(hipStream_t s, int64_t E, const MixedElem* el, Tables1D* const* tabs,
                                 const double* params, const double* x, double* y, int max_n, int max_nd) {
    if (E <= 0) return hipSuccess;
    const size_t lds = ((size_t)max_nd + 3 * (size_t)max_n * max_n) * sizeof(double);
    const int grid = (int)(E < 65536 ? E : 65536);
    hipLaunchKernelGGL(k_mixed_operator, dim3(grid), dim3(256), lds, s, E, el, tabs, params, x, y);
    return hipGetLastError();
}

}  // namespace kp
