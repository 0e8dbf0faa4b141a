// Apply of the Kronecker-sum inverse for n = 16 on the matrix cores (Alg. 6 / Alg. 8).
//
// Two kernels, one workgroup of four waves per work item:
//
// k_apply16 (2D; a work item is an element and a group of up to 16
// right-hand sides).  The data is a 16 x 16 x 16 tensor X[a][b][c] held in
// LDS (updated in place) with padded pitches (c: 1, b: 17, a: 273) so that
// every access pattern below hits distinct banks; a runs over the right-hand
// sides and b, c are the x, y axes.  Every contraction out = M (x)_axis X is a
// 16 x 16 x 256 matrix product done as 16 tiles of 16 x 16 x 16 (M on the A
// side, the tensor read from LDS on the B side).  The quasi-triangular
// Sylvester solve T1 Y + Y T2^T = F runs over the columns j of the last axis
// from 15 to 0; each step is the product N_j [F[:, :, j]] batched over the
// slices a (plus T1 [.] products for the 2 x 2 blocks of T2) and a rank-1
// update of the remaining columns.  The fragments come from the
// fragment-ordered tables.
//
// k_apply16r3 (3D; a work item is an element and one right-hand side).  The
// tensor lives in registers (see the description above the kernel): MFMA
// outputs are fed straight back as operands, the axes are routed by choosing
// the operand side, and two LDS transposes move the third axis.  Its
// fragments are read from the row-major tables.
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

constexpr int kSB = 17;         // pitch of b
constexpr int kSA = 16 * 17 + 1;  // pitch of a
constexpr int kTensor = 16 * kSA;

__device__ __forceinline__ int xidx(int a, int b, int c) { return a * kSA + b * kSB + c; }

// The right-hand sides s0 .. s0 + 15 of a 2D element (256 entries each,
// contiguous from rs0): thread tid loads the entry pairs t = 2 (tid + 256 i),
// i < 8, as 16-byte loads through a buffer descriptor that ends at the
// element's last right-hand side, so the rows past it read zero with no
// condition and every load is in flight before the first wait.
constexpr int kBufWord3 = 0x00020000;  // raw buffer descriptor, word 3 (gfx9, 32-bit format)
struct Rhs16 {
    double2 v[8];
};
__device__ __forceinline__ Rhs16 load_rhs16(const double* rs0, int ns, int tid) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)rs0, (short)0, ns * 2048, kBufWord3);
    Rhs16 x;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        x.v[i] = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rs, 16 * (tid + 256 * i), 0, 0));
    return x;
}
template <class T>
__device__ __forceinline__ void store_rhs16(const Rhs16& x, T* X, int tid) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int t = 2 * (tid + 256 * i);
        X[xidx(t >> 8, (t >> 4) & 15, t & 15)] = (T)x.v[i].x;
        X[xidx(t >> 8, (t >> 4) & 15, (t & 15) + 1)] = (T)x.v[i].y;
    }
}

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
// A fragment: the lane's share of a 16 x 16 matrix A on the A side of the MFMA;
// mma(frag, B) returns the lane's four outputs D[orow(g, v)][c] of D = A B,
// where g = lane / 16, c = lane % 16 and B(k, j) reads the B side.
struct PolF32 {
    typedef float T;
    typedef float Tab;
    typedef floatx4 Acc;
    typedef Arr4<float> Vec;  // one register tile: the lane's four values
    __device__ __forceinline__ static int orow(int g, int v) { return 4 * g + v; }
    struct Frag { float a[4]; };
    typedef float FragTab;
    static constexpr int kFragStride = 1;  // element stride of the fragment tables, in ne units
    __device__ __forceinline__ static float tab(const Tab* t, int i) { return t[i]; }
    __device__ __forceinline__ static Frag load(const Tab* M, int g, int c) {
        Frag f;
        for (int kk = 0; kk < 4; ++kk) f.a[kk] = M[c * 16 + 4 * kk + g];
        return f;
    }
    __device__ __forceinline__ static Frag load_frag(const FragTab* F, int m, int l) {
        const float4 v = ((const float4*)F)[m * 64 + l];
        Frag f;
        f.a[0] = v.x; f.a[1] = v.y; f.a[2] = v.z; f.a[3] = v.w;
        return f;
    }
    template <class B>
    __device__ __forceinline__ static Acc mma(const Frag& f, B b, int g, int c) {
        Acc acc = {0.f, 0.f, 0.f, 0.f};
        for (int kk = 0; kk < 4; ++kk)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(f.a[kk], (float)b(4 * kk + g, c), acc, 0, 0, 0);
        return acc;
    }
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
    typedef double FragTab;
    static constexpr int kFragStride = 1;
    __device__ __forceinline__ static double tab(const Tab* t, int i) { return t[i]; }
    __device__ __forceinline__ static Frag load(const Tab* M, int g, int c) {
        Frag f;
        for (int kk = 0; kk < 4; ++kk) f.a[kk] = M[c * 16 + 4 * kk + g];
        return f;
    }
    __device__ __forceinline__ static Frag load_frag(const FragTab* F, int m, int l) {
        const double2* p = (const double2*)(F + (m * 64 + l) * 4);
        const double2 u = p[0], v = p[1];
        Frag f;
        f.a[0] = u.x; f.a[1] = u.y; f.a[2] = v.x; f.a[3] = v.y;
        return f;
    }
    template <class B>
    __device__ __forceinline__ static Acc mma(const Frag& f, B b, int g, int c) {
        Acc acc = {0.0, 0.0, 0.0, 0.0};
        for (int kk = 0; kk < 4; ++kk)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(f.a[kk], (double)b(4 * kk + g, c), acc, 0, 0, 0);
        return acc;
    }
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
    typedef uint16_t FragTab;
    static constexpr int kFragStride = 1;
    __device__ __forceinline__ static float tab(const Tab* t, int i) { return bf16_to_f32(t[i]); }
    __device__ __forceinline__ static Frag load(const Tab* M, int g, int c) {
        Frag f;
        for (int i = 0; i < 4; ++i) f.a[i] = (short)M[c * 16 + 4 * g + i];
        return f;
    }
    __device__ __forceinline__ static Frag load_frag(const FragTab* F, int m, int l) {
        Frag f;
        f.a = *(const shortx4*)(F + (m * 64 + l) * 4);
        return f;
    }
    template <class B>
    __device__ __forceinline__ static Acc mma(const Frag& f, B b, int g, int c) {
        shortx4 bb;
        for (int i = 0; i < 4; ++i) bb[i] = bf16s((float)b(4 * g + i, c));
        Acc acc = {0.f, 0.f, 0.f, 0.f};
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(f.a, bb, acc, 0, 0, 0);
    }
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
    typedef uint16_t FragTab;
    static constexpr int kFragStride = 2;
    __device__ __forceinline__ static float tab(const Tab* t, int i) { return t[i]; }
    __device__ __forceinline__ static Frag load_frag(const FragTab* F, int m, int l) {
        Frag f;
        f.hi = *(const shortx4*)(F + ((m * 2 + 0) * 64 + l) * 4);
        f.lo = *(const shortx4*)(F + ((m * 2 + 1) * 64 + l) * 4);
        return f;
    }
    __device__ __forceinline__ static void split(float v, short* h, short* l) {
        *h = bf16s(v);
        *l = bf16s(v - bf16_to_f32((uint16_t)*h));
    }
    __device__ __forceinline__ static Frag load(const Tab* M, int g, int c) {
        Frag f;
        for (int i = 0; i < 4; ++i) {
            short h, l;
            split(M[c * 16 + 4 * g + i], &h, &l);
            f.hi[i] = h;
            f.lo[i] = l;
        }
        return f;
    }
    template <class B>
    __device__ __forceinline__ static Acc mma(const Frag& f, B b, int g, int c) {
        shortx4 bh, bl;
        for (int i = 0; i < 4; ++i) {
            short h, l;
            split((float)b(4 * g + i, c), &h, &l);
            bh[i] = h;
            bl[i] = l;
        }
        Acc acc = {0.f, 0.f, 0.f, 0.f};
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(f.lo, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(f.hi, bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(f.hi, bh, acc, 0, 0, 0);
        return acc;
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

// ----------------------------------------------------------- building blocks
// X <- M (x)_axis X in place, axis in {0, 1, 2} of X[a][b][c].  Wave wv owns
// the column tiles t = wv, wv+4, wv+8, wv+12; all reads finish (barrier)
// before any write.  SKIP: tiles t >= nt are all zero and stay so (2D: the
// slices past the work item's last right-hand side) and are skipped (the
// rank-3 series; the rank-2 2D apply keeps all sixteen, which measured faster:
// skipping raised its FP32 registers 111 -> 152 and cost a wave per SIMD).
template <class P, int AXIS, bool SKIP = false>
__device__ __forceinline__ void contract(const typename P::Frag& f, typename P::T* X, int g, int c,
                                         int wv, int nt = 16) {
    typename P::Acc acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int t = wv + 4 * i;
        if (SKIP && t >= nt) continue;
        if (AXIS == 0)
            acc[i] = P::mma(f, [&](int k, int j) { return X[xidx(k, t, j)]; }, g, c);
        else if (AXIS == 1)
            acc[i] = P::mma(f, [&](int k, int j) { return X[xidx(t, k, j)]; }, g, c);
        else
            acc[i] = P::mma(f, [&](int k, int j) { return X[xidx(t, j, k)]; }, g, c);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int t = wv + 4 * i;
        if (SKIP && t >= nt) continue;
        for (int v = 0; v < 4; ++v) {
            if (AXIS == 0)
                X[xidx(P::orow(g, v), t, c)] = acc[i][v];
            else if (AXIS == 1)
                X[xidx(t, P::orow(g, v), c)] = acc[i][v];
            else
                X[xidx(t, c, P::orow(g, v))] = acc[i][v];
        }
    }
    __syncthreads();
}

// T1 Y + Y T2^T = F on every slice a (T1 on b, T2 on c), in place: column j of
// F is replaced by y_j once every wave has read it (it is not read again).
// Nf: fragments of N_0..N_15 staged in LDS; fT1: fragment of T1; kd: kinds of
// T2's diagonal blocks; T2s: T2 in LDS.  Wave 0 writes the solution columns;
// wave wv updates the remaining columns k = wv mod 4.
template <class P>
__device__ __forceinline__ void sylvester(const typename P::FragTab* Nf, const typename P::Frag& fT1,
                                          const int* kd, const typename P::T* T2s, typename P::T* F,
                                          int g, int c, int l, int wv) {
    typedef typename P::T T;
    bool skip = false;
#pragma clang loop unroll(full)
    for (int j = 15; j >= 0; --j) {
        if (skip) {
            skip = false;
            continue;
        }
        if (j >= 1 && kd[j] == 2) {
            const int j1 = j - 1;
            const T p = T2s[j * 16 + j];
            const T q = T2s[j1 * 16 + j];
            const T s = T2s[j * 16 + j1];
            typename P::Acc a1 = P::mma(fT1, [&](int k, int col) { return F[xidx(col, k, j1)]; }, g, c);
            typename P::Acc a2 = P::mma(fT1, [&](int k, int col) { return F[xidx(col, k, j)]; }, g, c);
            T h1[4], h2[4];
            for (int v = 0; v < 4; ++v) {
                const T g1 = F[xidx(c, P::orow(g, v), j1)], g2 = F[xidx(c, P::orow(g, v), j)];
                h1[v] = (T)a1[v] + p * g1 - q * g2;
                h2[v] = (T)a2[v] + p * g2 - s * g1;
            }
            __syncthreads();
            if (wv == 0)
                for (int v = 0; v < 4; ++v) {
                    F[xidx(c, P::orow(g, v), j1)] = h1[v];
                    F[xidx(c, P::orow(g, v), j)] = h2[v];
                }
            __syncthreads();
            const typename P::Frag fn = P::load_frag(Nf, j, l);
            typename P::Acc y1 = P::mma(fn, [&](int k, int col) { return F[xidx(col, k, j1)]; }, g, c);
            typename P::Acc y2 = P::mma(fn, [&](int k, int col) { return F[xidx(col, k, j)]; }, g, c);
            for (int k = wv; k < j1; k += 4) {
                const T ta = T2s[k * 16 + j1], tb = T2s[k * 16 + j];
                for (int v = 0; v < 4; ++v)
                    F[xidx(c, P::orow(g, v), k)] -= ta * (T)y1[v] + tb * (T)y2[v];
            }
            __syncthreads();
            if (wv == 0)
                for (int v = 0; v < 4; ++v) {
                    F[xidx(c, P::orow(g, v), j1)] = y1[v];
                    F[xidx(c, P::orow(g, v), j)] = y2[v];
                }
            skip = true;
        } else {
            const typename P::Frag fn = P::load_frag(Nf, j, l);
            // B(k, col) = F[a = col][b = k][j]; output Y[b' = orow(g, v)][a = c]
            typename P::Acc y = P::mma(fn, [&](int k, int col) { return F[xidx(col, k, j)]; }, g, c);
            for (int k = wv; k < j; k += 4) {
                const T t2 = T2s[k * 16 + j];
                for (int v = 0; v < 4; ++v) F[xidx(c, P::orow(g, v), k)] -= t2 * (T)y[v];
            }
            __syncthreads();
            if (wv == 0)
                for (int v = 0; v < 4; ++v) F[xidx(c, P::orow(g, v), j)] = y[v];
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- kernel
// DIM 3: work item = (element, rhs); DIM 2: work item = (element, group of up
// to 16 right-hand sides), the slices a being the right-hand sides.
// LDS: the tensor (in place), T2, and the fragments of N_0..N_15.
template <class P, int DIM, class Z = double>
__global__ void __launch_bounds__(256) k_apply16(int64_t E, int nrhs, const typename P::Tab* tabs,
                                                 int64_t tab_stride,
                                                 const typename P::FragTab* frags,
                                                 const int8_t* kinds, const double* r, Z* z) {
    typedef typename P::T T;
    typedef typename P::FragTab FT;
    extern __shared__ __align__(16) unsigned char smem[];
    T* X = (T*)smem;
    T* T2s = X + kTensor;
    FT* Nf = (FT*)(T2s + 256);
    constexpr int kNfEntries = 16 * 64 * 4 * P::kFragStride;  // FT entries of N_0..N_15
    const int tid = threadIdx.x, l = tid & 63, wv = tid >> 6, g = l >> 4, c = l & 15;
    const int groups = DIM == 3 ? nrhs : (nrhs + 15) / 16;
    const int64_t work = E * groups;
    for (int64_t w = blockIdx.x; w < work; w += gridDim.x) {
        const int64_t e = w / groups;
        const int grp = (int)(w % groups);
        const typename P::Tab* tab = tabs + e * tab_stride;
        const FT* fr = frags + e * tab_stride * P::kFragStride;
        // All global loads of the element are issued before the first LDS
        // write (a load followed by its store in one loop iteration would wait
        // for each load in turn): fragments of L0..L2, R0, R1 and T1 stay in
        // registers; N_0..N_15, T2 and the right-hand side go to LDS.
        typename P::Frag fL[5];
#pragma unroll
        for (int m = 0; m < 5; ++m) fL[m] = P::load_frag(fr, m, l);
        const typename P::Frag fT1 = P::load_frag(fr, 5, l);
        constexpr int n16 = kNfEntries * (int)sizeof(FT) / 16;  // 16-byte chunks of N_0..N_15
        static_assert(n16 % 256 == 0, "N fragments: whole 16-byte chunks per thread");
        uint4 nbuf[n16 / 256];
        {
            const uint4* src = (const uint4*)(fr + 7 * 64 * 4 * P::kFragStride);
#pragma unroll
            for (int i = 0; i < n16 / 256; ++i) nbuf[i] = src[tid + 256 * i];
        }
        double2 rbuf[8];
        Rhs16 rh;
        if (DIM == 3) {
            const double2* rw = (const double2*)(r + w * 4096);
#pragma unroll
            for (int i = 0; i < 8; ++i) rbuf[i] = rw[tid + 256 * i];
        } else {
            const int s0 = grp * 16;
            rh = load_rhs16(r + (e * nrhs + s0) * 256, nrhs - s0 < 16 ? nrhs - s0 : 16, tid);
        }
        const T t2v = (T)P::tab(tab + 6 * 256, tid);
        int kd[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) kd[j] = kinds[e * kMaxN + j];
        {
            uint4* dst = (uint4*)Nf;
#pragma unroll
            for (int i = 0; i < n16 / 256; ++i) dst[tid + 256 * i] = nbuf[i];
        }
        T2s[tid] = t2v;
        if (DIM == 3) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int t = 2 * (tid + 256 * i);
                X[xidx(t >> 8, (t >> 4) & 15, t & 15)] = (T)rbuf[i].x;
                X[xidx(t >> 8, (t >> 4) & 15, (t & 15) + 1)] = (T)rbuf[i].y;
            }
        } else {
            store_rhs16(rh, X, tid);
        }
        __syncthreads();
        if (DIM == 3) {
            contract<P, 0>(fL[0], X, g, c, wv);
            contract<P, 1>(fL[1], X, g, c, wv);
            contract<P, 2>(fL[2], X, g, c, wv);
        } else {
            contract<P, 1>(fL[0], X, g, c, wv);
            contract<P, 2>(fL[1], X, g, c, wv);
        }
        sylvester<P>(Nf, fT1, kd, T2s, X, g, c, l, wv);
        contract<P, 1>(fL[3], X, g, c, wv);
        contract<P, 2>(fL[4], X, g, c, wv);
        if (DIM == 3) {
            Z* zw = z + w * 4096;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int t = 2 * (tid + 256 * i);
                zw[t] = (Z)X[xidx(t >> 8, (t >> 4) & 15, t & 15)];
                zw[t + 1] = (Z)X[xidx(t >> 8, (t >> 4) & 15, (t & 15) + 1)];
            }
        } else {
            const int s0 = grp * 16;
            for (int t = tid; t < 4096; t += 256) {
                const int a = t >> 8, s = s0 + a;
                if (s < nrhs) z[(e * nrhs + s) * 256 + (t & 255)] = (Z)X[xidx(a, (t >> 4) & 15, t & 15)];
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------- 2D rank 3 (three Kronecker terms)
// z = P3^{-1} r with P3 = P2 + A3 (x) B3 (P2 the first two terms, whose
// Schur-route inverse is the apply above): z = sum_k d_k with d_0 = P2^{-1} r
// and d_{k+1} = -P2^{-1} (A3 (x) B3) d_k, the Neumann series of
// (I + P2^{-1} (A3 (x) B3))^{-1} P2^{-1}, which converges when the spectral
// radius of P2^{-1} (A3 (x) B3) is below one (0.33 at most on the 2D p = 15
// blocks).  Every term costs one rank-2 apply and one Kronecker product on the
// matrix cores, with the element's tables, the 16 right-hand sides of the work
// item and the running sum in LDS; the series stops when every right-hand
// side's last term is at most tol times its sum.  A work item that has not
// met that within maxit terms (or has produced a non-finite value) sets
// flags[e] (cleared by the caller before the launch) for the per-element
// GMRES kernel to redo.
template <class P>
__device__ __forceinline__ typename P::Tab stage_tab(double v) {
    if constexpr (sizeof(typename P::Tab) == 2)
        return (typename P::Tab)bf16s((float)v);
    else
        return (typename P::Tab)v;
}

template <class P>
__global__ void __launch_bounds__(256) k_apply16_rank3(int64_t E, int nrhs, const typename P::Tab* tabs,
                                                       int64_t tab_stride, const typename P::FragTab* frags,
                                                       const int8_t* kinds, const double* factors,
                                                       const double* r, double* z, int maxit, double tol,
                                                       int8_t* flags) {
    typedef typename P::T T;
    typedef typename P::FragTab FT;
    typedef typename P::Tab TB;
    extern __shared__ __align__(16) unsigned char smem[];
    T* X = (T*)smem;
    T* T2s = X + kTensor;
    T* Zs = T2s + 256;                 // the running sum, 4096
    double* part = (double*)(Zs + 4096);  // 4 waves x 32 partial sums
    TB* M3 = (TB*)(part + 128);        // -A3 and B3, 512 entries
    FT* Nf = (FT*)(M3 + 512 + 8);
    constexpr int kNfEntries = 16 * 64 * 4 * P::kFragStride;
    const int tid = threadIdx.x, l = tid & 63, wv = tid >> 6, g = l >> 4, c = l & 15;
    const int groups = (nrhs + 15) / 16;
    const int64_t work = E * groups;
    for (int64_t w = blockIdx.x; w < work; w += gridDim.x) {
        const int64_t e = w / groups;
        const int grp = (int)(w % groups);
        const int s0 = grp * 16;
        const int ns = nrhs - s0 < 16 ? nrhs - s0 : 16;  // active slices
        const typename P::Tab* tab = tabs + e * tab_stride;
        const FT* fr = frags + e * tab_stride * P::kFragStride;
        typename P::Frag fL[5];
#pragma unroll
        for (int m = 0; m < 5; ++m) fL[m] = P::load_frag(fr, m, l);
        const typename P::Frag fT1 = P::load_frag(fr, 5, l);
        constexpr int n16 = kNfEntries * (int)sizeof(FT) / 16;
        uint4 nbuf[n16 / 256];
        {
            const uint4* src = (const uint4*)(fr + 7 * 64 * 4 * P::kFragStride);
#pragma unroll
            for (int i = 0; i < n16 / 256; ++i) nbuf[i] = src[tid + 256 * i];
        }
        const T t2v = (T)P::tab(tab + 6 * 256, tid);
        const double* F = factors + e * 6 * 256;
        const double a3 = F[4 * 256 + tid], b3 = F[5 * 256 + tid];
        int kd[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) kd[j] = kinds[e * kMaxN + j];
        const Rhs16 rh = load_rhs16(r + (e * nrhs + s0) * 256, ns, tid);
        {
            uint4* dst = (uint4*)Nf;
#pragma unroll
            for (int i = 0; i < n16 / 256; ++i) dst[tid + 256 * i] = nbuf[i];
        }
        T2s[tid] = t2v;
        M3[tid] = stage_tab<P>(-a3);
        M3[256 + tid] = stage_tab<P>(b3);
        store_rhs16(rh, X, tid);
#pragma unroll
        for (int i = 0; i < 16; ++i) Zs[tid + 256 * i] = (T)0;
        __syncthreads();
        const typename P::Frag fA3 = P::load(M3, g, c);
        const typename P::Frag fB3 = P::load(M3 + 256, g, c);
        bool done = false, ok = false;
        for (int it = 0; it < maxit && !done; ++it) {
            // d = P2^{-1} X
            contract<P, 1, true>(fL[0], X, g, c, wv, ns);
            contract<P, 2, true>(fL[1], X, g, c, wv, ns);
            sylvester<P>(Nf, fT1, kd, T2s, X, g, c, l, wv);
            contract<P, 1, true>(fL[3], X, g, c, wv, ns);
            contract<P, 2, true>(fL[4], X, g, c, wv, ns);
            // sum += d; per slice ||d||^2 and ||sum||^2 (thread tid holds entry
            // tid of every slice a = i)
            // one slice at a time, so that two partial sums are live, not 32
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int t = tid + 256 * i;
                const T dv = X[xidx(i, (t >> 4) & 15, t & 15)];
                const T zv = Zs[t] + dv;
                Zs[t] = zv;
                double pd = (double)dv * (double)dv;
                double pz = (double)zv * (double)zv;
                for (int off = 32; off > 0; off >>= 1) {
                    pd += __shfl_xor(pd, off, 64);
                    pz += __shfl_xor(pz, off, 64);
                }
                if (l == 0) {
                    part[wv * 32 + i] = pd;
                    part[wv * 32 + 16 + i] = pz;
                }
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
                done = ok = true;
                break;
            }
            // X = -(A3 (x) B3) d
            contract<P, 1, true>(fA3, X, g, c, wv, ns);
            contract<P, 2, true>(fB3, X, g, c, wv, ns);
        }
        for (int t = tid; t < 4096; t += 256) {
            const int a = t >> 8, sl = s0 + a;
            if (a < ns) z[(e * nrhs + sl) * 256 + (t & 255)] = (double)Zs[t];
        }
        if (tid == 0 && !ok) flags[e] = 1;
        __syncthreads();
    }
}

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
// The Neumann series of k_apply16_rank3 with the tensor and the element's
// fragments in registers (the running sum in LDS, one slot per thread).  Each later term
// d_{k+1} = -P2^{-1} (A3 (x) B3) d_k runs the rank-2 route of k_apply16r2
// with its first two products merged with the Kronecker factors: the L
// factor on y times B3 and the L factor on x times -A3, formed once per
// element on the matrix cores, so that a term costs one rank-2 apply and no
// more.  d_0 = P2^{-1} r takes the L factors alone.  The stopping test and
// the flags are those of k_apply16_rank3.

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

template <class P, int DIM, class Z>
static hipError_t launch16(hipStream_t st, int64_t E, int nrhs, const void* tabs, int64_t tab_stride,
                           const void* frags, const int8_t* kinds, const double* r, Z* z) {
    const int groups = DIM == 3 ? nrhs : (nrhs + 15) / 16;
    const int64_t work = E * groups;
    const int grid = (int)(work < kApply16Grid ? work : kApply16Grid);
    const size_t lds = (kTensor + 256) * sizeof(typename P::T) +
                       16 * 64 * 4 * P::kFragStride * sizeof(typename P::FragTab);
    hipLaunchKernelGGL((k_apply16<P, DIM, Z>), dim3(grid), dim3(256), lds, st, E, nrhs,
                       (const typename P::Tab*)tabs, tab_stride, (const typename P::FragTab*)frags,
                       kinds, r, z);
    return hipGetLastError();
}

template <class P>
static hipError_t launch16_rank3(hipStream_t st, int64_t E, int nrhs, const void* tabs, int64_t tab_stride,
                                 const void* frags, const int8_t* kinds, const double* factors, const double* r,
                                 double* z, int maxit, double tol, int8_t* flags) {
    const int64_t work = E * ((nrhs + 15) / 16);
    const int grid = (int)(work < kApply16Grid ? work : kApply16Grid);
    const size_t lds = (kTensor + 256 + 4096) * sizeof(typename P::T) + 128 * sizeof(double) +
                       (512 + 8) * sizeof(typename P::Tab) +
                       16 * 64 * 4 * P::kFragStride * sizeof(typename P::FragTab);
    hipLaunchKernelGGL((k_apply16_rank3<P>), dim3(grid), dim3(256), lds, st, E, nrhs,
                       (const typename P::Tab*)tabs, tab_stride, (const typename P::FragTab*)frags, kinds,
                       factors, r, z, maxit, tol, flags);
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
                                int64_t tab_stride, const void* frags, const int8_t* kinds,
                                const double* factors, const double* r, double* z, int8_t* flags, bool lds2d) {
    if (!lds2d && prec == 0)
        return launch16r2_rank3<PolF64, 2>(s, E, nrhs, tabs, tab_stride, kinds, factors, r, z, 256, 1e-14, flags);
    if (!lds2d && prec == 1)
        return launch16r2_rank3<PolF32, 4>(s, E, nrhs, tabs, tab_stride, kinds, factors, r, z, 128, 2e-7, flags);
    if (!lds2d && prec == 2)
        return launch16r2_rank3<PolBF16, 4>(s, E, nrhs, tabs, tab_stride, kinds, factors, r, z, 64, 2e-3, flags);
    if (!lds2d && prec == 3)
        return launch16r2_rank3<PolBF16X3, 3>(s, E, nrhs, tabs, tab_stride, kinds, factors, r, z, 96, 5e-6, flags);
    switch (prec) {
        // term limits: a spectral radius up to about 0.88 still converges within them
        case 0: return launch16_rank3<PolF64>(s, E, nrhs, tabs, tab_stride, frags, kinds, factors, r, z, 256, 1e-14,
                                              flags);
        case 1: return launch16_rank3<PolF32>(s, E, nrhs, tabs, tab_stride, frags, kinds, factors, r, z, 128, 2e-7,
                                              flags);
        case 2: return launch16_rank3<PolBF16>(s, E, nrhs, tabs, tab_stride, frags, kinds, factors, r, z, 64, 2e-3,
                                               flags);
        default: return launch16_rank3<PolBF16X3>(s, E, nrhs, tabs, tab_stride, frags, kinds, factors, r, z, 96,
                                                  5e-6, flags);
    }
}

hipError_t launch_apply16(hipStream_t s, int prec, int64_t E, int dim, int nrhs, const void* tabs,
                          int64_t tab_stride, const void* frags, const int8_t* kinds,
                          const double* r, double* z, const int8_t* axes, bool lds2d) {
    if (dim == 3) {
        switch (prec) {
            case 0: return launch16r3<PolF64, 2, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z, axes);
            case 1: return launch16r3<PolF32, 4, 7>(s, E, nrhs, tabs, tab_stride, kinds, r, z, axes);
            case 2: return launch16r3<PolBF16, 4, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z, axes);
            default: return launch16r3<PolBF16X3, 3, 7>(s, E, nrhs, tabs, tab_stride, kinds, r, z, axes);
        }
    }
    if (!lds2d) {
        switch (prec) {
            case 0: return launch16r2<PolF64, 2, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z);
            case 1: return launch16r2<PolF32, 4, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z);
            case 2: return launch16r2<PolBF16, 4, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z);
            default: return launch16r2<PolBF16X3, 3, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z);
        }
    }
    switch (prec) {
        case 0: return launch16<PolF64, 2>(s, E, nrhs, tabs, tab_stride, frags, kinds, r, z);
        case 1: return launch16<PolF32, 2>(s, E, nrhs, tabs, tab_stride, frags, kinds, r, z);
        case 2: return launch16<PolBF16, 2>(s, E, nrhs, tabs, tab_stride, frags, kinds, r, z);
        default: return launch16<PolBF16X3, 2>(s, E, nrhs, tabs, tab_stride, frags, kinds, r, z);
    }
}

hipError_t launch_apply16(hipStream_t s, int prec, int64_t E, int dim, int nrhs, const void* tabs,
                          int64_t tab_stride, const void* frags, const int8_t* kinds,
                          const double* r, float* z, const int8_t* axes, bool lds2d) {
    if (prec == 0) return hipErrorInvalidValue;  // FP64 arithmetic: z stays FP64
    if (dim == 3) {
        switch (prec) {
            case 1: return launch16r3<PolF32, 4, 7>(s, E, nrhs, tabs, tab_stride, kinds, r, z, axes);
            case 2: return launch16r3<PolBF16, 4, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z, axes);
            default: return launch16r3<PolBF16X3, 3, 7>(s, E, nrhs, tabs, tab_stride, kinds, r, z, axes);
        }
    }
    if (!lds2d) {
        switch (prec) {
            case 1: return launch16r2<PolF32, 4, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z);
            case 2: return launch16r2<PolBF16, 4, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z);
            default: return launch16r2<PolBF16X3, 3, 0>(s, E, nrhs, tabs, tab_stride, kinds, r, z);
        }
    }
    switch (prec) {
        case 1: return launch16<PolF32, 2>(s, E, nrhs, tabs, tab_stride, frags, kinds, r, z);
        case 2: return launch16<PolBF16, 2>(s, E, nrhs, tabs, tab_stride, frags, kinds, r, z);
        default: return launch16<PolBF16X3, 2>(s, E, nrhs, tabs, tab_stride, frags, kinds, r, z);
    }
}

}  // namespace kp
