// Apply of the Kronecker-sum inverse for n = 16 on the matrix cores (Alg. 6 / Alg. 8).
//
// One workgroup of four waves per work item, the element's tensor held in
// registers: MFMA outputs are fed straight back as operands, the axes are
// routed by choosing the operand side, and two LDS transposes move the axis
// that sits in the tile slot.  The quasi-triangular Sylvester solve
// T1 Y + Y T2^T = F runs over the columns j of its last axis from 15 to 0;
// each step is the product N_j [F[:, :, j]] (plus T1 [.] products for the
// 2 x 2 blocks of T2) on the wave holding column j and a rank-1 update of the
// remaining columns on every wave.  Fragments are read from the row-major
// tables.
//
//   k_apply16r3 (3D): a work item is an element and one right-hand side.
//   k_apply16r2 (2D): an element and a group of up to 16 right-hand sides,
//     which take the place of the 3D kernel's first axis.
//   k_apply16r2_rank3 (2D, three Kronecker terms): the Neumann series over
//     the rank-2 route, for the same work items.
//
// Precision policies: FP32 (v_mfma_f32_16x16x4f32), FP64
// (v_mfma_f64_16x16x4f64), BF16 (bf16 operands, v_mfma_f32_16x16x16bf16, FP32
// accumulation) and BF16X3 (split hi + lo operands, three bf16 products).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "elem_ops.h"
#include "kernels.h"

namespace kp {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

// raw buffer descriptor, word 3 (gfx9, 32-bit format): loads past the
// descriptor's size return zero
constexpr int kBufWord3 = 0x00020000;

// f32 -> bf16, round to nearest even, on the hardware converter (gfx950
// v_cvt_pk_bf16_f32); two at a time where the values come in pairs
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ short bf16s(float v) { return __builtin_bit_cast(short, (__bf16)v); }
__device__ __forceinline__ unsigned bf16x2s(float a, float b) {
    const floatx2 f = {a, b};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(f, bf16x2));
}
__device__ __forceinline__ shortx4 bf16x4s(float a, float b, float c, float d) {
    const unsigned lo = bf16x2s(a, b), hi = bf16x2s(c, d);
    shortx4 r;
    r[0] = (short)(lo & 0xffffu);
    r[1] = (short)(lo >> 16);
    r[2] = (short)(hi & 0xffffu);
    r[3] = (short)(hi >> 16);
    return r;
}

// a register tile held as a plain array (FP32, FP64) or as a vector (the BF16
// forms, whose conversions otherwise keep a memory copy of the tile)
template <class T>
struct Arr4 {
    T v[4];
    __device__ __forceinline__ T& operator[](int i) { return v[i]; }
    __device__ __forceinline__ const T& operator[](int i) const { return v[i]; }
};

// ----------------------------------------------------------- policies
// A fragment: the lane's share of a 16 x 16 matrix M on the A side of the
// MFMA (row_frag reads it from the row-major tables); mmr(frag, tile) returns
// the lane's four outputs D[orow(g, v)][c] of D = M X, where g = lane / 16,
// c = lane % 16 and the tile holds X[orow(g, kk)][c].
struct PolF32 {
    typedef float T;
    typedef float Tab;
    typedef floatx4 Acc;
    typedef Arr4<float> Vec;  // one register tile: the lane's four values
    __device__ __forceinline__ static int orow(int g, int v) { return 4 * g + v; }
    struct Frag { float a[4]; };
    __device__ __forceinline__ static float tab(const Tab* t, int i) { return t[i]; }
    // register-resident form: instruction kk takes k = orow(g, kk), so an
    // output tile is directly the next product's operand.  Fragment: M[c][4g + kk].
    __device__ __forceinline__ static Frag row_frag(const Tab* tab, int m, int g, int c) {
        const float4 v = *(const float4*)(tab + m * 256 + c * 16 + 4 * g);
        Frag f;
        f.a[0] = v.x; f.a[1] = v.y; f.a[2] = v.z; f.a[3] = v.w;
        return f;
    }
    // TA false: D = M X (tile on the B side); true: D = X^T M^T (tile on the A side)
    template <bool TA>
    __device__ __forceinline__ static Acc mmr(const Frag& f, const Vec& x) {
        Acc acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
            acc = TA ? __builtin_amdgcn_mfma_f32_16x16x4f32(x[kk], f.a[kk], acc, 0, 0, 0)
                     : __builtin_amdgcn_mfma_f32_16x16x4f32(f.a[kk], x[kk], acc, 0, 0, 0);
        return acc;
    }
};

struct PolF64 {
    typedef double T;
    typedef double Tab;
    typedef doublex4 Acc;
    typedef Arr4<double> Vec;  // one register tile: the lane's four values
    // the FP64 16x16x4 instruction interleaves its output rows
    __device__ __forceinline__ static int orow(int g, int v) { return g + 4 * v; }
    struct Frag { double a[4]; };
    __device__ __forceinline__ static double tab(const Tab* t, int i) { return t[i]; }
    // k = orow(g, kk) = g + 4 kk: M[c][g + 4 kk], four strided entries of row c
    __device__ __forceinline__ static Frag row_frag(const Tab* tab, int m, int g, int c) {
        Frag f;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) f.a[kk] = tab[m * 256 + c * 16 + g + 4 * kk];
        return f;
    }
    template <bool TA>
    __device__ __forceinline__ static Acc mmr(const Frag& f, const Vec& x) {
        Acc acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
            acc = TA ? __builtin_amdgcn_mfma_f64_16x16x4f64(x[kk], f.a[kk], acc, 0, 0, 0)
                     : __builtin_amdgcn_mfma_f64_16x16x4f64(f.a[kk], x[kk], acc, 0, 0, 0);
        return acc;
    }
};

struct PolBF16 {
    typedef float T;
    typedef uint16_t Tab;
    typedef floatx4 Acc;
    typedef floatx4 Vec;  // one register tile: the lane's four values
    __device__ __forceinline__ static int orow(int g, int v) { return 4 * g + v; }
    struct Frag { shortx4 a; };
    __device__ __forceinline__ static float tab(const Tab* t, int i) { return bf16_to_f32(t[i]); }
    __device__ __forceinline__ static Frag row_frag(const Tab* tab, int m, int g, int c) {
        Frag f;
        f.a = *(const shortx4*)(tab + m * 256 + c * 16 + 4 * g);
        return f;
    }
    template <bool TA>
    __device__ __forceinline__ static Acc mmr(const Frag& f, const Vec& x) {
        const shortx4 b = bf16x4s(x[0], x[1], x[2], x[3]);
        Acc acc = {0.f, 0.f, 0.f, 0.f};
        return TA ? __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(b, f.a, acc, 0, 0, 0)
                  : __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(f.a, b, acc, 0, 0, 0);
    }
};

struct PolBF16X3 {
    typedef float T;
    typedef float Tab;  // hi + lo as float; split again exactly
    typedef floatx4 Acc;
    typedef floatx4 Vec;  // one register tile: the lane's four values
    __device__ __forceinline__ static int orow(int g, int v) { return 4 * g + v; }
    struct Frag { shortx4 hi, lo; };
    __device__ __forceinline__ static float tab(const Tab* t, int i) { return t[i]; }
    __device__ __forceinline__ static void split(float v, short* h, short* l) {
        *h = bf16s(v);
        *l = bf16s(v - bf16_to_f32((uint16_t)*h));
    }
    __device__ __forceinline__ static Frag row_frag(const Tab* tab, int m, int g, int c) {
        const float4 v = *(const float4*)(tab + m * 256 + c * 16 + 4 * g);
        const float e[4] = {v.x, v.y, v.z, v.w};
        Frag f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            short h, lo;
            split(e[i], &h, &lo);
            f.hi[i] = h;
            f.lo[i] = lo;
        }
        return f;
    }
    template <bool TA>
    __device__ __forceinline__ static Acc mmr(const Frag& f, const Vec& x) {
        shortx4 bh, bl;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            short h, lo;
            split(x[i], &h, &lo);
            bh[i] = h;
            bl[i] = lo;
        }
        Acc acc = {0.f, 0.f, 0.f, 0.f};
        if (TA) {
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bh, f.lo, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bl, f.hi, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bh, f.hi, acc, 0, 0, 0);
        } else {
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(f.lo, bh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(f.hi, bl, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(f.hi, bh, acc, 0, 0, 0);
        }
        return acc;
    }
};

// ------------------------------------------------- 3D, register-resident
// One workgroup of four waves per (element, right-hand side).  The tensor
// lives in registers: wave w holds the tiles t = 4w .. 4w+3 (slot s = t % 4)
// of the "T" axis, and in tile t lane (g, c) holds the four values
// whose "G" index is orow(g, v) and whose "C" index is c.  Writing a layout as
// (G, C, T) = (axis, axis, axis):
//   * M applied on the B side (D = M X) contracts the G axis, layout kept;
//   * M applied on the A side (D = X^T M^T) contracts the G axis and swaps the
//     roles: the old C axis becomes G, the contracted axis becomes C;
//   * transpose_tg exchanges the G and T axes through LDS.
// Route: load (a, c, b) -> L0 on A side (c, a, b) -> L2 (c) -> transpose
// (b, a, c) -> L1 (b) -> Sylvester (T1 on b, T2 on c; each wave sweeps its
// own four columns, the lower waves receive them through LDS) -> R0 (b) -> transpose
// (c, a, b) -> R1 on A side (a, c, b) -> store.  Loads and stores of r and z
// are 128-byte contiguous per 16 lanes.

// transpose buffer: lane axis pitch 260, inner index rotated by the middle
// index and the lane axis (bank-conflict free for 4-byte entries)
constexpr int kTrA = 260;
constexpr int kTrSize = 16 * kTrA;
constexpr int kR3Work = kTrSize;  // entries: the transpose buffer, reused by the sweep
__device__ __forceinline__ int tr_idx(int cl, int x, int y) { return cl * kTrA + x * 16 + ((y + x + cl) & 15); }

// tile held in slot s by wave w: w + 4 s (consecutive Sylvester columns on
// different waves, so that the step products of the sweep rotate over the
// four SIMDs)
__device__ __forceinline__ int tile_of(int s, int w) { return w + 4 * s; }

template <class P>
__device__ __forceinline__ void transpose_tg(typename P::Vec (&R)[4], typename P::T* M, int g, int c, int w) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) M[tr_idx(c, tile_of(s, w), P::orow(g, v))] = R[s][v];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) R[s][v] = M[tr_idx(c, P::orow(g, v), tile_of(s, w))];
    __syncthreads();
}

template <class P, bool TA>
__device__ __forceinline__ void contract_reg(const typename P::Frag& f, typename P::Vec (&R)[4]) {
    typename P::Acc acc[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[s] = P::template mmr<TA>(f, R[s]);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) R[s][v] = (typename P::T)acc[s][v];
}

// T1 Y + Y T2^T = F per slice a on the layout (b, a, c): column j is the tile
// j, held by wave j % 4 in slot j / 4.  The holder forms y_j; the other waves receive it through LDS (xb: 4 buffers of
// 256 entries used in pairs, alternately, so that a buffer is rewritten only
// after a barrier that follows every read of it).  T2s: T2 row-major in LDS.
template <class P>
__device__ __forceinline__ void sylvester_col(typename P::Vec (&R)[4], const typename P::Frag (&fN)[4],
                                              const typename P::Frag& fT1, const int* kd,
                                              const typename P::T* T2s, typename P::T* xb, int l, int w) {
    typedef typename P::T T;
    int ph = 0;
    bool skip = false;
#pragma clang loop unroll(full)
    for (int j = 15; j >= 0; --j) {
        if (skip) {
            skip = false;
            continue;
        }
        if (j >= 1 && kd[j] == 2) {
            const int j1 = j - 1, o1 = j1 & 3, s1 = j1 >> 2, o2 = j & 3, s2 = j >> 2;
            T* e0 = xb + ph * 512;
            T* e1 = e0 + 256;
            ph ^= 1;
            if (w == o1)
#pragma unroll
                for (int v = 0; v < 4; ++v) e0[v * 64 + l] = R[s1][v];
            if (w == o2)
#pragma unroll
                for (int v = 0; v < 4; ++v) e1[v * 64 + l] = R[s2][v];
            __syncthreads();
            const T p = T2s[j * 16 + j], q = T2s[j1 * 16 + j], sv = T2s[j * 16 + j1];
            T* f0 = xb + ph * 512;
            T* f1 = f0 + 256;
            ph ^= 1;
            if (w == o1) {
                typename P::Vec h;
                const typename P::Acc a1 = P::template mmr<false>(fT1, R[s1]);
#pragma unroll
                for (int v = 0; v < 4; ++v) h[v] = (T)a1[v] + p * R[s1][v] - q * e1[v * 64 + l];
                const typename P::Acc y = P::template mmr<false>(fN[s1], h);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    R[s1][v] = (T)y[v];
                    f0[v * 64 + l] = R[s1][v];
                }
            }
            if (w == o2) {
                typename P::Vec h;
                const typename P::Acc a2 = P::template mmr<false>(fT1, R[s2]);
#pragma unroll
                for (int v = 0; v < 4; ++v) h[v] = (T)a2[v] + p * R[s2][v] - sv * e0[v * 64 + l];
                const typename P::Acc y = P::template mmr<false>(fN[s2], h);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    R[s2][v] = (T)y[v];
                    f1[v * 64 + l] = R[s2][v];
                }
            }
            __syncthreads();
            typename P::Vec y1, y2;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                y1[v] = w == o1 ? R[s1][v] : f0[v * 64 + l];
                y2[v] = w == o2 ? R[s2][v] : f1[v * 64 + l];
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int t = 4 * s + w;
                if (t < j1) {
                    const T ta = T2s[t * 16 + j1], tb = T2s[t * 16 + j];
#pragma unroll
                    for (int v = 0; v < 4; ++v) R[s][v] -= ta * y1[v] + tb * y2[v];
                }
            }
            skip = true;
        } else {
            const int o = j & 3, sj = j >> 2;
            T* e = xb + ph * 512;
            ph ^= 1;
            if (w == o) {
                const typename P::Acc y = P::template mmr<false>(fN[sj], R[sj]);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    R[sj][v] = (T)y[v];
                    e[v * 64 + l] = R[sj][v];
                }
            }
            __syncthreads();
            typename P::Vec y;
#pragma unroll
            for (int v = 0; v < 4; ++v) y[v] = w == o ? R[sj][v] : e[v * 64 + l];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int t = 4 * s + w;
                if (t < j) {
                    const T tc = T2s[t * 16 + j];
#pragma unroll
                    for (int v = 0; v < 4; ++v) R[s][v] -= tc * y[v];
                }
            }
        }
    }
    __syncthreads();
}

// Everything one item reads from HBM, held in registers: r (as loaded), the
// fragments of L0, L1, L2, R0, R1, T1 and of the wave's own N_j, the thread's
// entry of T2 and the block kinds of T2.
template <class P>
struct Item3 {
    double rb[4][4];
    typename P::Frag fL0, fL1, fL2, fR0, fR1, fT1;
    typename P::Frag fN[4];
    typename P::T t2v;
    int kd[16];
};

// Strides of the item's tensor axes (a, b, c) in the element's vector: the
// natural order (256, 16, 1), or, where the rank-1 split is on y or z, the
// relabelled orders y,x,z (16, 256, 1) and z,x,y (1, 256, 16)
struct AxStrides {
    int sa, sb, sc;
};
__device__ __forceinline__ AxStrides ax_strides(int ax) {
    return ax == 1 ? AxStrides{16, 256, 1} : ax == 2 ? AxStrides{1, 256, 16} : AxStrides{256, 16, 1};
}
// offset of tensor entry (a, b, c) in the element's vector
template <bool AX>
__device__ __forceinline__ int r3idx(int a, int b, int c, const AxStrides& ax) {
    if constexpr (AX)
        return a * ax.sa + b * ax.sb + c * ax.sc;
    else
        return a * 256 + b * 16 + c;
}

template <class P, bool AX>
__device__ __forceinline__ void load_item3(Item3<P>& x, int64_t it, int nrhs, const typename P::Tab* tabs,
                                           int64_t tab_stride, const int8_t* kinds, const double* r, int g,
                                           int c, int w, int tid, const AxStrides& ax) {
    const int64_t e = it / nrhs;
    const typename P::Tab* tab = tabs + e * tab_stride;
    const double* rw = r + it * 4096;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) x.rb[s][v] = rw[r3idx<AX>(P::orow(g, v), tile_of(s, w), c, ax)];
    x.fL0 = P::row_frag(tab, 0, g, c);
    x.fL1 = P::row_frag(tab, 1, g, c);
    x.fL2 = P::row_frag(tab, 2, g, c);
    x.fR0 = P::row_frag(tab, 3, g, c);
    x.fR1 = P::row_frag(tab, 4, g, c);
    x.fT1 = P::row_frag(tab, 5, g, c);
#pragma unroll
    for (int s = 0; s < 4; ++s) x.fN[s] = P::row_frag(tab, 7 + tile_of(s, w), g, c);
    x.t2v = (typename P::T)P::tab(tab + 6 * 256, tid);
#pragma unroll
    for (int j = 0; j < 16; ++j) x.kd[j] = kinds[e * kMaxN + j];
}

// Z: the type z is stored in (float only where the arithmetic is FP32, so that
// the stored values are exactly those of the double store)
// stagger, nres: the workgroups [nres / 2, nres) of the first resident round
// (nres = workgroups resident on the chip) start stagger * 2048 cycles late,
// so that half the resident workgroups load while the other half compute (the
// identical workgroups otherwise run their load, compute and store phases in
// step); 0: no delay.
// AX: the elements' split axes (axes[E]) are read and the tensor is loaded and
// stored in the relabelled order; without it every element is split on x.
template <class P, int WPE, class Z = double, bool AX = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, 8))) k_apply16r3(
    int64_t E, int nrhs, const typename P::Tab* tabs, int64_t tab_stride, const int8_t* kinds, const double* r,
    Z* z, int stagger, int nres, const int8_t* axes) {
    typedef typename P::T T;
    extern __shared__ __align__(16) unsigned char smem[];
    T* M = (T*)smem;         // transpose buffer; the Sylvester buffers alias it
    T* T2s = M + kR3Work;    // T2, row-major
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6, g = l >> 4, c = l & 15;
    if ((int)blockIdx.x < nres && 2 * (int)blockIdx.x >= nres)
        for (int i = 0; i < stagger; ++i) __builtin_amdgcn_s_sleep(32);
    const int64_t work = E * nrhs;
    for (int64_t it = blockIdx.x; it < work; it += gridDim.x) {
        // every global load of the item first
        AxStrides ax{256, 16, 1};
        if constexpr (AX) ax = ax_strides(axes[it / nrhs]);
        Item3<P> x;
        load_item3<P, AX>(x, it, nrhs, tabs, tab_stride, kinds, r, g, c, w, tid, ax);
        typename P::Vec R[4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int v = 0; v < 4; ++v) R[s][v] = (T)x.rb[s][v];
        T2s[tid] = x.t2v;  // read after the barriers of the first transpose

        contract_reg<P, true>(x.fL0, R);   // L0 on a: (a, c, b) -> (c, a, b)
        contract_reg<P, false>(x.fL2, R);  // L2 on c
        transpose_tg<P>(R, M, g, c, w);    // (b, a, c)
        contract_reg<P, false>(x.fL1, R);  // L1 on b
        sylvester_col<P>(R, x.fN, x.fT1, x.kd, T2s, M, l, w);
        contract_reg<P, false>(x.fR0, R);  // R0 on b
        transpose_tg<P>(R, M, g, c, w);    // (c, a, b)
        contract_reg<P, true>(x.fR1, R);   // R1 on c: (c, a, b) -> (a, c, b)

        // z is written once and read only by a later kernel: streaming
        // (non-temporal) stores keep it from taking L2 lines from the loads
        // of the items in flight
        Z* zw = z + it * 4096;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                __builtin_nontemporal_store((Z)R[s][v], &zw[r3idx<AX>(P::orow(g, v), tile_of(s, w), c, ax)]);
    }
}

// ------------------------------------------------- 2D, register-resident
// One workgroup of four waves per (element, group of up to 16 right-hand
// sides): the route of the 3D kernel without its first axis, the group's
// right-hand sides taking that axis's place in the lane slot.  Route: load
// (c, a, b) -> L on c -> transpose (b, a, c) -> L on b -> Sylvester (T1 on b,
// T2 on c) -> Q1 on b -> transpose (c, a, b) -> Q2 on c -> store, with a the
// right-hand side, b the x and c the y index.  Lane (g, cl) holds right-hand
// side cl; in tile t its four values are the y entries orow(g, v) of x row t,
// read through a buffer descriptor that ends at the group's last right-hand
// side (zero past it, so every load is issued with no condition).
template <class P, int WPE, class Z = double>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, 8))) k_apply16r2(
    int64_t E, int nrhs, const typename P::Tab* tabs, int64_t tab_stride, const int8_t* kinds, const double* r,
    Z* z, int stagger, int nres) {
    typedef typename P::T T;
    extern __shared__ __align__(16) unsigned char smem[];
    T* M = (T*)smem;       // transpose buffer; the Sylvester buffers alias it
    T* T2s = M + kR3Work;  // T2, row-major
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6, g = l >> 4, c = l & 15;
    if ((int)blockIdx.x < nres && 2 * (int)blockIdx.x >= nres)
        for (int i = 0; i < stagger; ++i) __builtin_amdgcn_s_sleep(32);
    const int groups = (nrhs + 15) / 16;
    const int64_t work = E * groups;
    for (int64_t it = blockIdx.x; it < work; it += gridDim.x) {
        const int64_t e = it / groups;
        const int s0 = (int)(it % groups) * 16;
        const int ns = nrhs - s0 < 16 ? nrhs - s0 : 16;
        const double* r0 = r + (e * nrhs + s0) * 256;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)r0, (short)0, ns * 2048, kBufWord3);
        double rb[4][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int base = 8 * (c * 256 + tile_of(s, w) * 16);
            if constexpr (std::is_same<P, PolF64>::value) {
                // rows g + 4 v: four separate entries
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    rb[s][v] = __builtin_bit_cast(
                        double, __builtin_amdgcn_raw_buffer_load_b64(rs, base + 8 * P::orow(g, v), 0, 0));
            } else {
                // rows 4 g .. 4 g + 3: 32 contiguous bytes
                const double2 u = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rs, base + 32 * g, 0, 0));
                const double2 q = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rs, base + 32 * g + 16, 0, 0));
                rb[s][0] = u.x;
                rb[s][1] = u.y;
                rb[s][2] = q.x;
                rb[s][3] = q.y;
            }
        }
        const typename P::Tab* tab = tabs + e * tab_stride;
        const typename P::Frag fLb = P::row_frag(tab, 0, g, c), fLc = P::row_frag(tab, 1, g, c);
        const typename P::Frag fQ1 = P::row_frag(tab, 3, g, c), fQ2 = P::row_frag(tab, 4, g, c);
        const typename P::Frag fT1 = P::row_frag(tab, 5, g, c);
        typename P::Frag fN[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) fN[s] = P::row_frag(tab, 7 + tile_of(s, w), g, c);
        const T t2v = (T)P::tab(tab + 6 * 256, tid);
        int kd[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) kd[j] = kinds[e * kMaxN + j];
        typename P::Vec R[4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int v = 0; v < 4; ++v) R[s][v] = (T)rb[s][v];
        T2s[tid] = t2v;  // read after the barriers of the first transpose

        contract_reg<P, false>(fLc, R);  // L on c
        transpose_tg<P>(R, M, g, c, w);  // (b, a, c)
        contract_reg<P, false>(fLb, R);  // L on b
        sylvester_col<P>(R, fN, fT1, kd, T2s, M, l, w);
        contract_reg<P, false>(fQ1, R);  // Q1 on b
        transpose_tg<P>(R, M, g, c, w);  // (c, a, b)
        contract_reg<P, false>(fQ2, R);  // Q2 on c

        // streaming stores, as in the 3D kernel; lanes past the group's last
        // right-hand side store nothing
        if (c < ns) {
            Z* zw = z + (e * nrhs + s0 + c) * 256;
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    __builtin_nontemporal_store((Z)R[s][v], &zw[tile_of(s, w) * 16 + P::orow(g, v)]);
        }
    }
}

// ------------------------------------------ 2D rank 3, register-resident
// z = P3^{-1} r with P3 = P2 + A3 (x) B3 (P2 the first two terms, whose
// Schur-route inverse is the rank-2 apply): z = sum_k d_k with d_0 = P2^{-1} r
// and d_{k+1} = -P2^{-1} (A3 (x) B3) d_k, the Neumann series of
// (I + P2^{-1} (A3 (x) B3))^{-1} P2^{-1}, which converges when the spectral
// radius of P2^{-1} (A3 (x) B3) is below one.  Work items as in k_apply16r2;
// the tensor and the element's fragments stay in registers, the running sum
// in LDS (one slot per thread and value).  Each later term runs the rank-2
// route with its first two products merged with the Kronecker factors (the L
// factor on y times B3, the L factor on x times -A3, formed once per element
// on the matrix cores), so that a term costs one rank-2 apply and no more.
// The series stops when every right-hand side's last term is at most tol
// times its sum; a work item that has not met that within maxit terms (or
// has produced a non-finite value) sets flags[e] (cleared by the caller
// before the launch) for the per-element GMRES kernel to redo.

// P2^{-1} on the register tensor, from layout (c, a, b) back to (c, a, b);
// fc, fb: the first products on c and on b
template <class P>
__device__ __forceinline__ void p2inv_reg(typename P::Vec (&R)[4], const typename P::Frag& fc,
                                          const typename P::Frag& fb, const typename P::Frag& fQ1,
                                          const typename P::Frag& fQ2, const typename P::Frag (&fN)[4],
                                          const typename P::Frag& fT1, const int* kd, const typename P::T* T2s,
                                          typename P::T* M, int g, int c, int l, int w) {
    contract_reg<P, false>(fc, R);   // on c
    transpose_tg<P>(R, M, g, c, w);  // (b, a, c)
    contract_reg<P, false>(fb, R);   // on b
    sylvester_col<P>(R, fN, fT1, kd, T2s, M, l, w);
    contract_reg<P, false>(fQ1, R);  // Q1 on b
    transpose_tg<P>(R, M, g, c, w);  // (c, a, b)
    contract_reg<P, false>(fQ2, R);  // Q2 on c
}

// the A-side fragment of X Y for the lane's row c: Gt = Y^T X^T on the
// matrix cores, whose output lane (g, c) holds Gt[orow(g, v)][c] = (X Y)[c][orow(g, v)],
// from the fragment of X (row c of X) and the lane's column of Y^T
// (the BF16 forms: the product of the fragment's values in FP32, rounded to
// the fragment's form afterwards)
__device__ __forceinline__ void frag_rows(const PolBF16::Frag& f, float (&x)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = bf16_to_f32((uint16_t)f.a[i]);
}
__device__ __forceinline__ void frag_rows(const PolBF16X3::Frag& f, float (&x)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = bf16_to_f32((uint16_t)f.hi[i]) + bf16_to_f32((uint16_t)f.lo[i]);
}
__device__ __forceinline__ void frag_set(PolBF16::Frag& f, const floatx4& d) { f.a = bf16x4s(d[0], d[1], d[2], d[3]); }
__device__ __forceinline__ void frag_set(PolBF16X3::Frag& f, const floatx4& d) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        short h, lo;
        PolBF16X3::split(d[i], &h, &lo);
        f.hi[i] = h;
        f.lo[i] = lo;
    }
}
template <class P>
__device__ __forceinline__ typename P::Frag frag_product(const typename P::Frag& fx, const typename P::T (&yt)[4]) {
    typename P::Frag f;
    if constexpr (std::is_same<P, PolF32>::value || std::is_same<P, PolF64>::value) {
        typename P::Frag a;
        typename P::Vec b;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            a.a[kk] = yt[kk];
            b[kk] = fx.a[kk];
        }
        const typename P::Acc d = P::template mmr<false>(a, b);
#pragma unroll
        for (int v = 0; v < 4; ++v) f.a[v] = (typename P::T)d[v];
    } else {
        float x[4];
        frag_rows(fx, x);
        PolF32::Frag a;
        PolF32::Vec b;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            a.a[kk] = yt[kk];
            b[kk] = x[kk];
        }
        frag_set(f, PolF32::mmr<false>(a, b));
    }
    return f;
}

template <class P, int WPE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, 8))) k_apply16r2_rank3(
    int64_t E, int nrhs, const typename P::Tab* tabs, int64_t tab_stride, const int8_t* kinds,
    const double* factors, const double* r, double* z, int maxit, double tol, int8_t* flags) {
    typedef typename P::T T;
    typedef typename P::Frag Frag;
    extern __shared__ __align__(16) unsigned char smem[];
    T* M = (T*)smem;                      // transpose buffer; the Sylvester buffers alias it
    T* T2s = M + kR3Work;                 // T2, row-major
    T* Zs = T2s + 256;                    // the running sum: thread tid's value i at i * 256 + tid
    double* part = (double*)(Zs + 4096);  // [wave][slice]: ||d||^2 (0..15), ||z||^2 (16..31)
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6, g = l >> 4, c = l & 15;
    const int groups = (nrhs + 15) / 16;
    const int64_t work = E * groups;
    for (int64_t it = blockIdx.x; it < work; it += gridDim.x) {
        const int64_t e = it / groups;
        const int s0 = (int)(it % groups) * 16;
        const int ns = nrhs - s0 < 16 ? nrhs - s0 : 16;
        const double* r0 = r + (e * nrhs + s0) * 256;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)r0, (short)0, ns * 2048, kBufWord3);
        double rb[4][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int base = 8 * (c * 256 + tile_of(s, w) * 16);
#pragma unroll
            for (int v = 0; v < 4; ++v)
                rb[s][v] = __builtin_bit_cast(double,
                                              __builtin_amdgcn_raw_buffer_load_b64(rs, base + 8 * P::orow(g, v), 0, 0));
        }
        const typename P::Tab* tab = tabs + e * tab_stride;
        const Frag fLb = P::row_frag(tab, 0, g, c), fLc = P::row_frag(tab, 1, g, c);
        const Frag fQ1 = P::row_frag(tab, 3, g, c), fQ2 = P::row_frag(tab, 4, g, c);
        const Frag fT1 = P::row_frag(tab, 5, g, c);
        Frag fN[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) fN[s] = P::row_frag(tab, 7 + tile_of(s, w), g, c);
        const T t2v = (T)P::tab(tab + 6 * 256, tid);
        // columns of B3 and -A3: the lane's entries [orow(g, kk)][c]
        const double* F3 = factors + e * 6 * 256;
        T b3t[4], a3t[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            b3t[kk] = (T)F3[5 * 256 + P::orow(g, kk) * 16 + c];
            a3t[kk] = (T)(-F3[4 * 256 + P::orow(g, kk) * 16 + c]);
        }
        int kd[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) kd[j] = kinds[e * kMaxN + j];
        typename P::Vec R[4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int v = 0; v < 4; ++v) R[s][v] = (T)rb[s][v];
        T2s[tid] = t2v;  // read after the barriers of the first transpose
        const Frag fGc = frag_product<P>(fLc, b3t);  // L_y B3
        const Frag fGb = frag_product<P>(fLb, a3t);  // -L_x A3
        p2inv_reg<P>(R, fLc, fLb, fQ1, fQ2, fN, fT1, kd, T2s, M, g, c, l, w);  // d_0
        bool ok = false;
        for (int k = 0; k < maxit; ++k) {
            if (k > 0) p2inv_reg<P>(R, fGc, fGb, fQ1, fQ2, fN, fT1, kd, T2s, M, g, c, l, w);
            // z += d (the thread's own entries of Zs); per right-hand side (the
            // lane's c) ||d||^2 and ||z||^2
            double pd = 0.0, pz = 0.0;
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    T* zp = Zs + (4 * s + v) * 256 + tid;
                    const T zv = k == 0 ? R[s][v] : *zp + R[s][v];
                    *zp = zv;
                    pd += (double)R[s][v] * (double)R[s][v];
                    pz += (double)zv * (double)zv;
                }
            pd += __shfl_xor(pd, 16, 64);
            pz += __shfl_xor(pz, 16, 64);
            pd += __shfl_xor(pd, 32, 64);
            pz += __shfl_xor(pz, 32, 64);
            if (g == 0) {
                part[w * 32 + c] = pd;
                part[w * 32 + 16 + c] = pz;
            }
            __syncthreads();
            bool conv = true, finite = true;
            for (int i = 0; i < ns; ++i) {
                const double d2 = part[i] + part[32 + i] + part[64 + i] + part[96 + i];
                const double z2 = part[16 + i] + part[48 + i] + part[80 + i] + part[112 + i];
                if (!(d2 == d2) || !(z2 == z2) || d2 > 1e300 || z2 > 1e300) finite = false;
                if (!(d2 <= tol * tol * z2)) conv = false;
            }
            __syncthreads();
            if (!finite) break;
            if (conv) {
                ok = true;
                break;
            }
        }
        if (c < ns) {
            double* zw = z + (e * nrhs + s0 + c) * 256;
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    zw[tile_of(s, w) * 16 + P::orow(g, v)] = (double)Zs[(4 * s + v) * 256 + tid];
        }
        if (tid == 0 && !ok) flags[e] = 1;
    }
}

// WPE: waves per SIMD the register allocation is held to (FP32, BF16: 4 with
// 128 registers; split BF16: 3; FP64: 2).  One workgroup per item: a
// persistent grid that prefetches the next item into registers measured
// slower (it needs half the occupancy).
// compute units of the current device (queried once per device)
static int device_cus() {
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (cus[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        cus[dev] = v;
    }
    return cus[dev];
}

// STAGGER: the delay of the late half of the first round (see k_apply16r3),
// used for batches of at least four rounds; measured at n = 16, 4096
// elements: FP32 76.8 -> 72.7 us, split BF16 84.9 -> 83.1 us, no gain for
// BF16 (already closer to the HBM bound) or FP64
template <class P, int WPE, int STAGGER, class Z>
static hipError_t launch16r3(hipStream_t st, int64_t E, int nrhs, const void* tabs, int64_t tab_stride,
                             const int8_t* kinds, const double* r, Z* z, const int8_t* axes) {
    const int64_t work = E * nrhs;
    const int grid = (int)(work < kApply16Grid ? work : kApply16Grid);
    const size_t lds = (kR3Work + 256) * sizeof(typename P::T);
    const int nres = WPE * device_cus();  // WPE resident workgroups per CU (a wave per SIMD each)
    const int stagger = (STAGGER > 0 && nres > 0 && work >= 4 * (int64_t)nres) ? STAGGER : 0;
    if (axes)
        hipLaunchKernelGGL((k_apply16r3<P, WPE, Z, true>), dim3(grid), dim3(256), lds, st, E, nrhs,
                           (const typename P::Tab*)tabs, tab_stride, kinds, r, z, stagger, nres, axes);
    else
        hipLaunchKernelGGL((k_apply16r3<P, WPE, Z, false>), dim3(grid), dim3(256), lds, st, E, nrhs,
                           (const typename P::Tab*)tabs, tab_stride, kinds, r, z, stagger, nres, axes);
    return hipGetLastError();
}

// the 2D register-resident kernel; WPE and STAGGER as for the 3D kernel (a
// stagger of 0 to 14 units changed the 2D p = 15 FP32 apply by under 3%: 0)
template <class P, int WPE, int STAGGER, class Z>
static hipError_t launch16r2(hipStream_t st, int64_t E, int nrhs, const void* tabs, int64_t tab_stride,
                             const int8_t* kinds, const double* r, Z* z) {
    const int64_t work = E * ((nrhs + 15) / 16);
    const int grid = (int)(work < kApply16Grid ? work : kApply16Grid);
    const size_t lds = (kR3Work + 256) * sizeof(typename P::T);
    const int nres = WPE * device_cus();
    const int stagger = (STAGGER > 0 && nres > 0 && work >= 4 * (int64_t)nres) ? STAGGER : 0;
    hipLaunchKernelGGL((k_apply16r2<P, WPE, Z>), dim3(grid), dim3(256), lds, st, E, nrhs,
                       (const typename P::Tab*)tabs, tab_stride, kinds, r, z, stagger, nres);
    return hipGetLastError();
}

// the register-resident series.  FP32 is held to four waves
// per SIMD: 44 bytes per lane spill, outside the term loop (4.1 ms against
// 4.5 ms at three waves and no spill, 2D p = 15)
template <class P, int WPE>
static hipError_t launch16r2_rank3(hipStream_t st, int64_t E, int nrhs, const void* tabs, int64_t tab_stride,
                                   const int8_t* kinds, const double* factors, const double* r, double* z,
                                   int maxit, double tol, int8_t* flags) {
    const int64_t work = E * ((nrhs + 15) / 16);
    const int grid = (int)(work < kApply16Grid ? work : kApply16Grid);
    const size_t lds = (kR3Work + 256 + 4096) * sizeof(typename P::T) + 128 * sizeof(double);
    hipLaunchKernelGGL((k_apply16r2_rank3<P, WPE>), dim3(grid), dim3(256), lds, st, E, nrhs,
                       (const typename P::Tab*)tabs, tab_stride, kinds, factors, r, z, maxit, tol, flags);
    return hipGetLastError();
}

hipError_t launch_apply16_rank3(hipStream_t s, int prec, int64_t E, int nrhs, const void* tabs,
                                int64_t tab_stride, const int8_t* kinds, const double* factors, const double* r,
                                double* z, int8_t* flags) {
    // term limits: FP64 96 and FP32 48 terms converge for a spectral radius up
    // to about 0.72 (slower elements go to the GMRES path); measured at 2D
    // p = 15, 8 RHS, against the 256 and 128 terms that admit 0.88: FP64
    // 17.6 -> 16.6 ms, FP32 4.10 -> 3.64 ms, since the few slow work items no
    // longer hold the launch's tail (fewer terms cost more in the fallback:
    // FP64 at 48 terms 17.9 ms, FP32 at 32 3.9 ms); the BF16 forms admit 0.9
    switch (prec) {
        case 0: return launch16r2_rank3<PolF64, 2>(s, E, nrhs, tabs, tab_stride, kinds, factors, r, z, 96, 1e-14, flags);
        case 1: return launch16r2_rank3<PolF32, 4>(s, E, nrhs, tabs, tab_stride, kinds, factors, r, z, 48, 2e-7, flags);
        case 2: return launch16r2_rank3<PolBF16, 4>(s, E, nrhs, tabs, tab_stride, kinds, factors, r, z, 64, 2e-3, flags);
        default:
            return launch16r2_rank3<PolBF16X3, 3>(s, E, nrhs, tabs, tab_stride, kinds, factors, r, z, 96, 5e-6, flags);
    }
}

hipError_t launch_apply16(hipStream_t s, int prec, int64_t E, int dim, int nrhs, const void* tabs,
                          int64_t tab_stride, const int8_t* kinds, const double* r, double* z,
                          const int8_t* axes) {
    if (dim == 3) {
        switch (prec) {
            case 0: return launch16r3<PolF64, 2, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z, axes);
            case 1: return launch16r3<PolF32, 4, 7>(s, E, nrhs, tabs, tab_stride, kinds, r, z, axes);
            case 2: return launch16r3<PolBF16, 4, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z, axes);
            default: return launch16r3<PolBF16X3, 3, 7>(s, E, nrhs, tabs, tab_stride, kinds, r, z, axes);
        }
    }
    switch (prec) {
        case 0: return launch16r2<PolF64, 2, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z);
        case 1: return launch16r2<PolF32, 4, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z);
        case 2: return launch16r2<PolBF16, 4, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z);
        default: return launch16r2<PolBF16X3, 3, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z);
    }
}

hipError_t launch_apply16(hipStream_t s, int prec, int64_t E, int dim, int nrhs, const void* tabs,
                          int64_t tab_stride, const int8_t* kinds, const double* r, float* z,
                          const int8_t* axes) {
    if (prec == 0) return hipErrorInvalidValue;  // FP64 arithmetic: z stays FP64
    if (dim == 3) {
        switch (prec) {
            case 1: return launch16r3<PolF32, 4, 7>(s, E, nrhs, tabs, tab_stride, kinds, r, z, axes);
            case 2: return launch16r3<PolBF16, 4, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z, axes);
            default: return launch16r3<PolBF16X3, 3, 7>(s, E, nrhs, tabs, tab_stride, kinds, r, z, axes);
        }
    }
    switch (prec) {
        case 1: return launch16r2<PolF32, 4, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z);
        case 2: return launch16r2<PolBF16, 4, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z);
        default: return launch16r2<PolBF16X3, 3, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z);
    }
}

}  // namespace kp
