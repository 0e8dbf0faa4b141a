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
// third word of a raw buffer descriptor on gfx9 (32-bit data format); raw
// buffer loads past the descriptor's byte count return zero
constexpr int kBufWord3 = 0x00020000;

// type of the tables' LDS copy: BF16 entries are held as FP32
template <typename TT>
struct SmallLdsTab {
    typedef TT type;
};
template <>
struct SmallLdsTab<uint16_t> {
    typedef float type;
};

__host__ __device__ inline size_t small3_wave_bytes(int n, size_t tsz, size_t tabsz) {
    const size_t tabs = ((size_t)(7 + n) * n * n * tabsz + 15) / 16 * 16;
    // the relayout buffer and the sweep's exchange blocks are never live at
    // the same time: one region serves both
    const size_t buf = (size_t)n * n * (n + 1), ex = 6 * (size_t)kS3 * kS3;
    return (tabs + (buf > ex ? buf : ex) * tsz + 15) / 16 * 16;
}

// NT: n fixed at compile time (0: n_arg), so that every fibre loop and
// table index folds to constants
template <typename T, typename TT, class Rnd, class Z, bool AX, int NT>
__global__ void __launch_bounds__(256) k_apply_small3(int64_t E, int n_arg, int nrhs, const TT* tabs,
                                                      int64_t tab_stride, const int8_t* kinds, const double* r, Z* z,
                                                      Rnd rnd, const int8_t* axes) {
    const int n = NT > 0 ? NT : n_arg;
    extern __shared__ __align__(16) unsigned char smem[];
    // the wave index as a scalar, so that the item index and every per-item
    // address below are scalars
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), l = (int)(threadIdx.x & 63);
    const int nn = n * n, nd = nn * n, n1 = n + 1;
    const int ntab = (7 + n) * nn;
    // the wave's copy of the tables in LDS: BF16 tables are widened to FP32
    // on the way in (exactly), so that no table read converts
    typedef typename SmallLdsTab<TT>::type LT;
    const size_t per = small3_wave_bytes(n, sizeof(T), sizeof(LT));
    LT* tb = (LT*)(smem + wv * per);
    T* buf = (T*)((unsigned char*)tb + ((size_t)ntab * sizeof(LT) + 15) / 16 * 16);
    T* ex = buf;            // six exchange blocks of kS3 x kS3 (slice, row), during the sweep
    const LT* L0 = tb;
    const LT* L1 = tb + nn;
    const LT* L2 = tb + 2 * nn;
    const LT* R0 = tb + 3 * nn;
    const LT* R1 = tb + 4 * nn;
    const LT* T1 = tb + 5 * nn;
    const LT* T2 = tb + 6 * nn;
    const LT* N = tb + 7 * nn;
    const bool act = l < nn;
    const int p = act ? l / n : 0, q = act ? l % n : 0;
    WaveTeam wt;
    // x <- M x along the fibre (M n x n row-major in LDS)
    auto inl = [&](const LT* M, T (&x)[kS3]) {
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
    // the tables are copied as 4-byte words: (7 + n) n^2 is even for every n,
    // so an element's tables start and end on a word boundary (the launcher
    // checks the stride)
    constexpr int kTabWords = ((7 + kS3) * kS3 * kS3 * (int)sizeof(TT) + 3) / 4;
    constexpr int kTabPer = (kTabWords + 63) / 64;
    const int nwords = ntab * (int)sizeof(TT) / 4;
    // buf, in units of one word's worth of LDS entries (a word, or two FP32
    // values for BF16 tables) from tb
    const int buf_unit = (int)(((size_t)ntab * sizeof(LT) + 15) / 16 * 16 / (4 * sizeof(LT) / sizeof(TT)));
    const int64_t work = E * nrhs;
    for (int64_t w = (int64_t)blockIdx.x * 4 + wv; w < work; w += (int64_t)gridDim.x * 4) {
        const int64_t e = w / nrhs;
        const TT* tabw = tabs + e * tab_stride;
        int sa = nn, sb = n, sc = 1;
        if (AX) {
            const int ax = axes[e];
            if (ax == 1) { sa = n; sb = nn; sc = 1; }
            else if (ax == 2) { sa = 1; sb = nn; sc = n; }
        }
        // every load of the item is issued before the first wait: the table
        // words, the r fibre and the block kinds of T2.  The tables and r are
        // read through buffer descriptors sized to the item, so a word past
        // the element's tables or a lane outside the element (its offset set
        // past the end) reads zero without touching memory.
        const __amdgpu_buffer_rsrc_t rt =
            __builtin_amdgcn_make_buffer_rsrc((void*)tabw, (short)0, nwords * 4, kBufWord3);
        uint32_t tv[kTabPer];
#pragma unroll
        for (int k = 0; k < kTabPer; ++k) tv[k] = __builtin_amdgcn_raw_buffer_load_b32(rt, 4 * l + 256 * k, 0, 0);
        const __amdgpu_buffer_rsrc_t rr =
            __builtin_amdgcn_make_buffer_rsrc((void*)(r + w * nd), (short)0, nd * 8, kBufWord3);
        const int lane_off = act ? 8 * (p * sb + q * sc) : (int)0x80000000;
        double rv[kS3];
#pragma unroll
        for (int f = 0; f < kS3; ++f)
            rv[f] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rr, lane_off + 8 * f * sa, 0, 0));
        // kinds of columns 0..7 (the section is 256-byte aligned, 32 bytes per element)
        const uint2 kdw = *(const uint2*)__builtin_assume_aligned(kinds + e * kMaxN, 8);
        // words past the tables go to the first word of the relayout buffer,
        // which is written before it is read (no branch, so that no load is
        // moved behind one)
#pragma unroll
        for (int k = 0; k < kTabPer; ++k) {
            const int id = l + 64 * k;
            const int dst = id < nwords ? id : buf_unit;
            if constexpr (sizeof(TT) == 2) {
                // the word's two BF16 entries, low half first
                const float2 v = {bf16_to_f32((uint16_t)(tv[k] & 0xffffu)), bf16_to_f32((uint16_t)(tv[k] >> 16))};
                ((float2*)tb)[dst] = v;
            } else {
                ((uint32_t*)tb)[dst] = tv[k];
            }
        }
        T x[kS3];
#pragma unroll
        for (int f = 0; f < kS3; ++f) x[f] = f < n ? (T)rv[f] : (T)0;
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
            const int kd = (int)(((j < 4 ? kdw.x : kdw.y) >> (8 * (j & 3))) & 0xffu);
            if (kd != 2) {
                const LT* Nj = N + j * nn;
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
                const LT* Nj = N + j * nn;
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
    // word copies of the tables need word-aligned element strides, and the
    // kinds are read eight at a time
    if ((tab_stride * (int64_t)sizeof(TT)) % 4 != 0 || ((uintptr_t)tabs & 3) != 0 || ((uintptr_t)kinds & 7) != 0)
        return hipErrorInvalidValue;
    const int64_t work = E * nrhs;
    const int64_t wg = (work + 3) / 4;
    const int grid = (int)(wg < 65536 ? wg : 65536);
    const size_t lds = 4 * small3_wave_bytes(n, sizeof(T), sizeof(typename SmallLdsTab<TT>::type));
    if (axes)
        hipLaunchKernelGGL((k_apply_small3<T, TT, Rnd, Z, true, 0>), dim3(grid), dim3(256), lds, s, E, n, nrhs,
                           (const TT*)tabs, tab_stride, kinds, r, z, rnd, axes);
    else if (n == kS3)
        hipLaunchKernelGGL((k_apply_small3<T, TT, Rnd, Z, false, kS3>), dim3(grid), dim3(256), lds, s, E, n, nrhs,
                           (const TT*)tabs, tab_stride, kinds, r, z, rnd, axes);
    else
        hipLaunchKernelGGL((k_apply_small3<T, TT, Rnd, Z, false, 0>), dim3(grid), dim3(256), lds, s, E, n, nrhs,
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
