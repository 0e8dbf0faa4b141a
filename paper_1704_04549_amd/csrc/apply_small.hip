// Apply of the Kronecker-sum inverse for 3D elements with n <= 8 (Alg. 8):
// one wave per (element, right-hand side), four per workgroup, no workgroup
// barrier.  The n^3 tensor lives in registers as fibres: lane (p, q), p, q < n,
// holds the n values along one axis at a fixed pair of the other two, in one
// of three layouts
//   A: fibre over a at (b, c) = (p, q)
//   B: fibre over b at (a, c) = (p, q)
//   C: fibre over c at (a, b) = (p, q),
// so that a contraction along the fibre's axis is n x n multiply-adds within
// the lane (the matrix read from the wave's copy of the element's tables in
// LDS, the same address on every lane).  Layouts change through an LDS buffer
// (index ((a n + b)(n + 1) + c): rows padded so that every layout's accesses
// fall on distinct banks).  Route: load (A) -> L0 -> B -> L1 -> C -> L2 -> B ->
// quasi-triangular Sylvester sweep over the columns c (the step's column of
// every slice goes through LDS, lane (a, i) forms row i of the solution
// column, which goes back through LDS to the lanes (a, k < j)) -> R0 -> C ->
// R1 -> A -> store.  Operands are rounded as in the generic
// apply (Rnd), so the arithmetic per entry is the same.
#include <hip/hip_runtime.h>

#include "elem_ops.h"
#include "kernels.h"

namespace kp {

constexpr int kS3 = 8;  // largest n of this kernel

__host__ __device__ inline size_t small3_wave_bytes(int n, size_t tsz, size_t tabsz) {
    const size_t tabs = ((size_t)(7 + n) * n * n * tabsz + 15) / 16 * 16;
    // the relayout buffer and the sweep's exchange blocks are never live at
    // the same time: one region serves both
    const size_t buf = (size_t)n * n * (n + 1), ex = 6 * (size_t)kS3 * kS3;
    return (tabs + (buf > ex ? buf : ex) * tsz + 15) / 16 * 16;
}

template <typename T, typename TT, class Rnd, class Z, bool AX>
__global__ void __launch_bounds__(256) k_apply_small3(int64_t E, int n, int nrhs, const TT* tabs, int64_t tab_stride,
                                                      const int8_t* kinds, const double* r, Z* z, Rnd rnd,
                                                      const int8_t* axes) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int wv = (int)(threadIdx.x >> 6), l = (int)(threadIdx.x & 63);
    const int nn = n * n, nd = nn * n, n1 = n + 1;
    const int ntab = (7 + n) * nn;
    const size_t per = small3_wave_bytes(n, sizeof(T), sizeof(TT));
    TT* tb = (TT*)(smem + wv * per);
    T* buf = (T*)((unsigned char*)tb + ((size_t)ntab * sizeof(TT) + 15) / 16 * 16);
    T* ex = buf;            // six exchange blocks of kS3 x kS3 (slice, row), during the sweep
    const TT* L0 = tb;
    const TT* L1 = tb + nn;
    const TT* L2 = tb + 2 * nn;
    const TT* R0 = tb + 3 * nn;
    const TT* R1 = tb + 4 * nn;
    const TT* T1 = tb + 5 * nn;
    const TT* T2 = tb + 6 * nn;
    const TT* N = tb + 7 * nn;
    const bool act = l < nn;
    const int p = act ? l / n : 0, q = act ? l % n : 0;
    WaveTeam wt;
    // x <- M x along the fibre (M n x n row-major in LDS)
    auto inl = [&](const TT* M, T (&x)[kS3]) {
        T xr[kS3], y[kS3];
#pragma unroll
        for (int k = 0; k < kS3; ++k) xr[k] = rnd(x[k]);
#pragma unroll
        for (int i = 0; i < kS3; ++i) {
            T acc = (T)0;
#pragma unroll
            for (int k = 0; k < kS3; ++k)
                if (i < n && k < n) acc += (T)ldt(M, i * n + k) * xr[k];
            y[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < kS3; ++i) x[i] = y[i];
    };
    // LDS index of tensor entry (a, b, c)
    auto pidx = [&](int a, int b, int c) { return (a * n + b) * n1 + c; };
    // fibre f of lane (p, q) in layout L is entry (a, b, c) =
    //   A: (f, p, q)   B: (p, f, q)   C: (p, q, f)
    auto relayout = [&](T (&x)[kS3], int from, int to) {
        if (act)
#pragma unroll
            for (int f = 0; f < kS3; ++f)
                if (f < n) {
                    const int id = from == 0 ? pidx(f, p, q) : from == 1 ? pidx(p, f, q) : pidx(p, q, f);
                    buf[id] = x[f];
                }
        wt.sync();
        if (act)
#pragma unroll
            for (int f = 0; f < kS3; ++f)
                if (f < n) {
                    const int id = to == 0 ? pidx(f, p, q) : to == 1 ? pidx(p, f, q) : pidx(p, q, f);
                    x[f] = buf[id];
                }
        wt.sync();
    };
    const int64_t work = E * nrhs;
    for (int64_t w = (int64_t)blockIdx.x * 4 + wv; w < work; w += (int64_t)gridDim.x * 4) {
        const int64_t e = w / nrhs;
        const TT* tab = tabs + e * tab_stride;
        for (int t = l; t < ntab; t += 64) tb[t] = tab[t];
        int sa = nn, sb = n, sc = 1;
        if (AX) {
            const int ax = axes[e];
            if (ax == 1) { sa = n; sb = nn; sc = 1; }
            else if (ax == 2) { sa = 1; sb = nn; sc = n; }
        }
        T x[kS3];
        const double* rw = r + w * nd;
#pragma unroll
        for (int f = 0; f < kS3; ++f) x[f] = (act && f < n) ? (T)rw[f * sa + p * sb + q * sc] : (T)0;
        wt.sync();
        // forward contractions: L0 on a (layout A), L1 on b (B), L2 on c (C)
        inl(L0, x);
        relayout(x, 0, 1);
        inl(L1, x);
        relayout(x, 1, 2);
        inl(L2, x);
        relayout(x, 2, 1);
        // Sylvester on every slice a = p: lane (p, q) holds column q of F (rows
        // b).  Each step's column products are spread over the lanes: lane
        // (a, i) forms row i of slice a's solution column from the column read
        // back from LDS, so every lane works in every step.
        T* xa = ex;                   // F column(s) of the step, per slice
        T* xb = ex + kS3 * kS3;
        T* ha = ex + 2 * kS3 * kS3;   // the 2 x 2 step's right-hand sides
        T* hb = ex + 3 * kS3 * kS3;
        T* ya = ex + 4 * kS3 * kS3;   // solution column(s) of the step
        T* yb = ex + 5 * kS3 * kS3;
        const int i = q;              // the row this lane forms
        int j = n - 1;
        while (j >= 0) {
            const int kd = kinds[e * kMaxN + j];
            if (kd != 2) {
                const TT* Nj = N + j * nn;
                if (act && q == j)
#pragma unroll
                    for (int k = 0; k < kS3; ++k)
                        if (k < n) xa[p * kS3 + k] = x[k];
                wt.sync();
                if (act) {
                    T acc = (T)0;
#pragma unroll
                    for (int k = 0; k < kS3; ++k)
                        if (k < n) acc += (T)ldt(Nj, i * n + k) * rnd(xa[p * kS3 + k]);
                    ya[p * kS3 + i] = acc;
                }
                wt.sync();
                if (act && q < j) {
                    const T t2 = (T)ldt(T2, q * n + j);
#pragma unroll
                    for (int k = 0; k < kS3; ++k)
                        if (k < n) x[k] -= t2 * rnd(ya[p * kS3 + k]);
                } else if (act && q == j) {
#pragma unroll
                    for (int k = 0; k < kS3; ++k)
                        if (k < n) x[k] = ya[p * kS3 + k];
                }
                wt.sync();
                --j;
            } else {
                const int j1 = j - 1;
                const T pp = (T)ldt(T2, j * n + j), qq = (T)ldt(T2, j1 * n + j), sv = (T)ldt(T2, j * n + j1);
                const TT* Nj = N + j * nn;
                if (act && (q == j1 || q == j)) {
                    T* dst = q == j1 ? xa : xb;
#pragma unroll
                    for (int k = 0; k < kS3; ++k)
                        if (k < n) dst[p * kS3 + k] = x[k];
                }
                wt.sync();
                // row i of h1 = (T1 + p I) g1 - q g2 and h2 = (T1 + p I) g2 - s g1
                if (act) {
                    T a1 = (T)0, a2 = (T)0;
#pragma unroll
                    for (int k = 0; k < kS3; ++k)
                        if (k < n) {
                            const T tk = (T)ldt(T1, i * n + k);
                            a1 += tk * rnd(xa[p * kS3 + k]);
                            a2 += tk * rnd(xb[p * kS3 + k]);
                        }
                    const T g1 = xa[p * kS3 + i], g2 = xb[p * kS3 + i];
                    ha[p * kS3 + i] = a1 + pp * g1 - qq * g2;
                    hb[p * kS3 + i] = a2 + pp * g2 - sv * g1;
                }
                wt.sync();
                if (act) {
                    T y1 = (T)0, y2 = (T)0;
#pragma unroll
                    for (int k = 0; k < kS3; ++k)
                        if (k < n) {
                            const T nk = (T)ldt(Nj, i * n + k);
                            y1 += nk * rnd(ha[p * kS3 + k]);
                            y2 += nk * rnd(hb[p * kS3 + k]);
                        }
                    ya[p * kS3 + i] = y1;
                    yb[p * kS3 + i] = y2;
                }
                wt.sync();
                if (act && q < j1) {
                    const T ta = (T)ldt(T2, q * n + j1), tbv = (T)ldt(T2, q * n + j);
#pragma unroll
                    for (int k = 0; k < kS3; ++k)
                        if (k < n) x[k] -= ta * rnd(ya[p * kS3 + k]) + tbv * rnd(yb[p * kS3 + k]);
                } else if (act && (q == j1 || q == j)) {
                    const T* src = q == j1 ? ya : yb;
#pragma unroll
                    for (int k = 0; k < kS3; ++k)
                        if (k < n) x[k] = src[p * kS3 + k];
                }
                wt.sync();
                j -= 2;
            }
        }
        // backward contractions: R0 on b (layout B), R1 on c (C)
        inl(R0, x);
        relayout(x, 1, 2);
        inl(R1, x);
        // store from layout A: for each a the wave writes n^2 consecutive values
        relayout(x, 2, 0);
        if (act) {
            Z* zw = z + w * nd;
#pragma unroll
            for (int f = 0; f < kS3; ++f)
                if (f < n) __builtin_nontemporal_store((Z)x[f], &zw[f * sa + p * sb + q * sc]);
        }
        wt.sync();  // the wave's tables and buffers are rewritten by its next item
    }
}

template <typename T, typename TT, class Rnd, class Z>
static hipError_t small3(hipStream_t s, int64_t E, int n, int nrhs, const void* tabs, int64_t tab_stride,
                         const int8_t* kinds, const double* r, Z* z, Rnd rnd, const int8_t* axes) {
    const int64_t work = E * nrhs;
    const int64_t wg = (work + 3) / 4;
    const int grid = (int)(wg < 65536 ? wg : 65536);
    const size_t lds = 4 * small3_wave_bytes(n, sizeof(T), sizeof(TT));
    if (axes)
        hipLaunchKernelGGL((k_apply_small3<T, TT, Rnd, Z, true>), dim3(grid), dim3(256), lds, s, E, n, nrhs,
                           (const TT*)tabs, tab_stride, kinds, r, z, rnd, axes);
    else
        hipLaunchKernelGGL((k_apply_small3<T, TT, Rnd, Z, false>), dim3(grid), dim3(256), lds, s, E, n, nrhs,
                           (const TT*)tabs, tab_stride, kinds, r, z, rnd, axes);
    return hipGetLastError();
}

template <class Z>
static hipError_t launch_small3(hipStream_t s, int prec, int64_t E, int n, int nrhs, const void* tabs,
                                int64_t tab_stride, const int8_t* kinds, const double* r, Z* z, const int8_t* axes) {
    if (n < 2 || n > kS3 || E <= 0 || nrhs <= 0) return E <= 0 || nrhs <= 0 ? hipSuccess : hipErrorInvalidValue;
    switch (prec) {
        case 0: return small3<double, double>(s, E, n, nrhs, tabs, tab_stride, kinds, r, z, RoundNone(), axes);
        case 1: return small3<float, float>(s, E, n, nrhs, tabs, tab_stride, kinds, r, z, RoundNone(), axes);
        case 2: return small3<float, uint16_t>(s, E, n, nrhs, tabs, tab_stride, kinds, r, z, RoundBf16(), axes);
        default: return small3<float, float>(s, E, n, nrhs, tabs, tab_stride, kinds, r, z, RoundBf16x2(), axes);
    }
}

hipError_t launch_apply_small3(hipStream_t s, int prec, int64_t E, int n, int nrhs, const void* tabs,
                               int64_t tab_stride, const int8_t* kinds, const double* r, double* z,
                               const int8_t* axes) {
    return launch_small3(s, prec, E, n, nrhs, tabs, tab_stride, kinds, r, z, axes);
}

hipError_t launch_apply_small3(hipStream_t s, int prec, int64_t E, int n, int nrhs, const void* tabs,
                               int64_t tab_stride, const int8_t* kinds, const double* r, float* z,
                               const int8_t* axes) {
    if (prec == 0) return hipErrorInvalidValue;  // FP64 arithmetic: z stays FP64
    return launch_small3(s, prec, E, n, nrhs, tabs, tab_stride, kinds, r, z, axes);
}

}  // namespace kp
