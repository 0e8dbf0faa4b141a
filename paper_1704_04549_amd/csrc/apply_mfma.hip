// Apply of the Kronecker-sum inverse for n = 16 on the matrix cores (Alg. 6 / Alg. 8).
//
// One workgroup of four waves per (element, slice group).  The element's data
// is a 16 x 16 x 16 tensor X[a][b][c] held in LDS (updated in place) with
// padded pitches (c: 1, b: 17, a: 273) so
// that every access pattern below (contiguous in c, strided by b or by a) hits
// distinct banks.  In 3D a, b, c are the x, y, z axes of one right-hand side;
// in 2D a runs over up to 16 right-hand sides and b, c are the x, y axes.
//
// Every contraction out = M (x)_axis X is a 16 x 16 x 256 matrix product done
// as 16 tiles of 16 x 16 x 16 on the MFMA units (M on the A side, the tensor
// on the B side, the two untouched axes spanning the columns).  The
// quasi-triangular Sylvester solve T1 Y + Y T2^T = F runs over the columns j
// of the last axis from 15 to 0; each step is the 16 x 16 x 16 product
// N_j [F[:, :, j]] batched over the slices a (plus T1 [.] products for the
// 2 x 2 blocks of T2), and a rank-1 update of the remaining columns.  The four
// waves split the 16 column tiles of every contraction; in the Sylvester sweep
// each wave forms the (small) step product itself and updates every fourth
// remaining column.
//
// Precision policies: FP32 (v_mfma_f32_16x16x4f32), FP64
// (v_mfma_f64_16x16x4f64), BF16 (bf16 operands, v_mfma_f32_16x16x16bf16, FP32
// accumulation) and BF16X3 (split hi + lo operands, three bf16 products).
#include <hip/hip_runtime.h>

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

__device__ __forceinline__ short bf16s(float v) { return (short)f32_to_bf16(v); }

// ----------------------------------------------------------- policies
// A fragment: the lane's share of a 16 x 16 matrix A on the A side of the MFMA;
// mma(frag, B) returns the lane's four outputs D[orow(g, v)][c] of D = A B,
// where g = lane / 16, c = lane % 16 and B(k, j) reads the B side.
struct PolF32 {
    typedef float T;
    typedef float Tab;
    typedef floatx4 Acc;
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
};

struct PolF64 {
    typedef double T;
    typedef double Tab;
    typedef doublex4 Acc;
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
};

struct PolBF16 {
    typedef float T;
    typedef uint16_t Tab;
    typedef floatx4 Acc;
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
};

struct PolBF16X3 {
    typedef float T;
    typedef float Tab;  // hi + lo as float; split again exactly
    typedef floatx4 Acc;
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
        const uint16_t hb = f32_to_bf16(v);
        *h = (short)hb;
        *l = bf16s(v - bf16_to_f32(hb));
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
};

// ----------------------------------------------------------- building blocks
// X <- M (x)_axis X in place, axis in {0, 1, 2} of X[a][b][c].  Wave wv owns
// the column tiles t = wv, wv+4, wv+8, wv+12; all reads finish (barrier)
// before any write.
template <class P, int AXIS>
__device__ __forceinline__ void contract(const typename P::Frag& f, typename P::T* X, int g, int c,
                                         int wv) {
    typename P::Acc acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int t = wv + 4 * i;
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
template <class P, int DIM>
__global__ void __launch_bounds__(256) k_apply16(int64_t E, int nrhs, const typename P::Tab* tabs,
                                                 int64_t tab_stride,
                                                 const typename P::FragTab* frags,
                                                 const int8_t* kinds, const double* r, double* z) {
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
        if (DIM == 3) {
            const double2* rw = (const double2*)(r + w * 4096);
#pragma unroll
            for (int i = 0; i < 8; ++i) rbuf[i] = rw[tid + 256 * i];
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
            const int s0 = grp * 16;
            for (int t = tid; t < 4096; t += 256) {
                const int a = t >> 8, s = s0 + a;
                X[xidx(a, (t >> 4) & 15, t & 15)] =
                    s < nrhs ? (T)r[(e * nrhs + s) * 256 + (t & 255)] : (T)0;
            }
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
            double2* zw = (double2*)(z + w * 4096);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int t = 2 * (tid + 256 * i);
                double2 v;
                v.x = (double)X[xidx(t >> 8, (t >> 4) & 15, t & 15)];
                v.y = (double)X[xidx(t >> 8, (t >> 4) & 15, (t & 15) + 1)];
                zw[tid + 256 * i] = v;
            }
        } else {
            const int s0 = grp * 16;
            for (int t = tid; t < 4096; t += 256) {
                const int a = t >> 8, s = s0 + a;
                if (s < nrhs) z[(e * nrhs + s) * 256 + (t & 255)] = (double)X[xidx(a, (t >> 4) & 15, t & 15)];
            }
        }
        __syncthreads();
    }
}

template <class P, int DIM>
static hipError_t launch16(hipStream_t st, int64_t E, int nrhs, const void* tabs, int64_t tab_stride,
                           const void* frags, const int8_t* kinds, const double* r, double* z) {
    const int groups = DIM == 3 ? nrhs : (nrhs + 15) / 16;
    const int64_t work = E * groups;
    const int grid = (int)(work < kApply16Grid ? work : kApply16Grid);
    const size_t lds = (kTensor + 256) * sizeof(typename P::T) +
                       16 * 64 * 4 * P::kFragStride * sizeof(typename P::FragTab);
    hipLaunchKernelGGL((k_apply16<P, DIM>), dim3(grid), dim3(256), lds, st, E, nrhs,
                       (const typename P::Tab*)tabs, tab_stride, (const typename P::FragTab*)frags,
                       kinds, r, z);
    return hipGetLastError();
}

hipError_t launch_apply16(hipStream_t s, int prec, int64_t E, int dim, int nrhs, const void* tabs,
                          int64_t tab_stride, const void* frags, const int8_t* kinds,
                          const double* r, double* z) {
    if (dim == 3) {
        switch (prec) {
            case 0: return launch16<PolF64, 3>(s, E, nrhs, tabs, tab_stride, frags, kinds, r, z);
            case 1: return launch16<PolF32, 3>(s, E, nrhs, tabs, tab_stride, frags, kinds, r, z);
            case 2: return launch16<PolBF16, 3>(s, E, nrhs, tabs, tab_stride, frags, kinds, r, z);
            default: return launch16<PolBF16X3, 3>(s, E, nrhs, tabs, tab_stride, frags, kinds, r, z);
        }
    }
    switch (prec) {
        case 0: return launch16<PolF64, 2>(s, E, nrhs, tabs, tab_stride, frags, kinds, r, z);
        case 1: return launch16<PolF32, 2>(s, E, nrhs, tabs, tab_stride, frags, kinds, r, z);
        case 2: return launch16<PolBF16, 2>(s, E, nrhs, tabs, tab_stride, frags, kinds, r, z);
        default: return launch16<PolBF16X3, 2>(s, E, nrhs, tabs, tab_stride, frags, kinds, r, z);
    }
}

}  // namespace kp
