// HIP kernels of the KSVD preconditioner for gfx950.
//
// Setup kernels run one element per workgroup with the team routines of
// elem_ops.h; the hot apply kernels for n = 16 live in apply_mfma.hip.
#include <hip/hip_runtime.h>

#include "elem_ops.h"
#include "kernels.h"
#include "mixed.h"

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
                                               int32_t status_or, const double* grams) {
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
        W.Gpre = grams ? grams + e * nn * nn : nullptr;
        int st = setup_element<kRefine>(tm, dim, n, rank, T, params + e * kRecLen, blk, g,
                               factors + e * nf * nn, sigma + e * 4, W, g2);
        if (threadIdx.x == 0) status[e] = st | status_or;
        __syncthreads();
    }
}

// One wave per element (four elements per workgroup, independent waves, no
// workgroup barrier inside the loop): each wave has its own workspace slot
// and its own LDS small arrays; the workgroup shares the 1D tables.
// Specialised on the dimension and on explicit / structured input, so that
// each instance carries only its own path (registers are sized for the
// longest path of an instance).
template <bool kRefine, int DIM, bool EXPL>
__global__ void __launch_bounds__(256) k_setup_waves(int64_t E, int dim_rt, int n, int rank,
                                                     const Tables1D* tab, const double* params,
                                                     const double* blocks, const double* guess,
                                                     double* factors, double* sigma, int32_t* status,
                                                     double* ws, int64_t ws_stride, const int32_t* skip,
                                                     int32_t status_or, int64_t small_stride,
                                                     const double* grams) {
    __shared__ Tables1D T;
    extern __shared__ double small[];
    {
        const double* src = (const double*)tab;
        double* dst = (double*)&T;
        for (int i = threadIdx.x; i < (int)(sizeof(Tables1D) / sizeof(double)); i += blockDim.x)
            dst[i] = src[i];
        __syncthreads();
    }
    (void)dim_rt;
    constexpr int dim = DIM;
    constexpr bool expl = EXPL;
    WaveTeam tm;
    const int wv = threadIdx.x >> 6;
    const int64_t slot = (int64_t)blockIdx.x * 4 + wv;
    SetupWork W = carve_setup_work(ws + slot * ws_stride, dim, n, expl, rank);
    carve_small(small + wv * small_stride, n, expl, &W);
    const long nn = (long)n * n;
    const long nd = dim == 2 ? nn : nn * n;
    const int nf = dim == 2 ? 2 * rank : 5;
    const long gs = dim == 3 ? 2 : 1;
    for (int64_t e = slot; e < E; e += (int64_t)gridDim.x * 4) {
        if (skip && skip[e]) continue;
        const double* blk = expl ? blocks + e * nd * nd : nullptr;
        const double* g = guess ? guess + e * gs * nn : nullptr;
        const double* g2 = (guess && dim == 3) ? g + nn : nullptr;
        W.Gpre = grams ? grams + e * nn * nn : nullptr;
        int st = setup_element<kRefine>(tm, DIM, n, rank, T, params + e * kRecLen, blk, g,
                                        factors + e * nf * nn, sigma + e * 4, W, g2);
        if ((threadIdx.x & 63) == 0) status[e] = st | status_or;
        tm.sync();
    }
}

// ---------------------------------------------------------- apply tables
// Where element q of a table launch lives: contiguous (list null: element q,
// factors at q fstride, tables at q tstride doubles) or, for a class of a
// mixed batch, element list[q] with the offsets of its descriptor.
struct TabAddr {
    const int32_t* list;
    const MixedElem* el;
    int64_t fstride, tstride;
    __device__ int64_t elem(int64_t q) const { return list ? (int64_t)list[q] : q; }
    __device__ int64_t fac(int64_t e) const { return list ? el[e].fac_off : e * fstride; }
    __device__ int64_t tab(int64_t e) const { return list ? el[e].tab_off : e * tstride; }
};

// Three kernels: prepare (one wave per element: pair rotation, inverses, C1
// and C2), Schur (one wave per (element, C matrix), with a small LDS
// footprint so that many run per CU) and finish (one wave per element: L
// tables, kinds, N_j).  Intermediates live in the element's own table slots.
__global__ void __launch_bounds__(64) k_tables_prepare(int64_t E, int dim, int n, int rank,
                                                       const double* factors, double* tab64,
                                                       int32_t* status, TabAddr ad) {
    extern __shared__ double lds[];
    __shared__ double red[kMaxReduce];
    __shared__ double sh[kMaxN + 8];
    __shared__ int ipiv[kMaxN];
    BlockTeam tm{red};
    const long nn = (long)n * n;
    const int nf = dim == 2 ? 2 * rank : 5;
    double* F = lds;              // nf n^2
    double* work = F + nf * nn;   // 10 n^2
    for (int64_t it = blockIdx.x; it < E; it += gridDim.x) {
        const int64_t e = ad.elem(it);
        for (long t = threadIdx.x; t < nf * nn; t += blockDim.x) F[t] = factors[ad.fac(e) + t];
        __syncthreads();
        double* tab = tab64 + ad.tab(e);
        const int st = tables_prepare(tm, dim, n, rank, F, tab, tab + 7 * nn, work, ipiv, sh);
        if (threadIdx.x == 0) status[e] |= st;
        __syncthreads();
    }
}

// Gauss-Jordan inverses of 64 / G matrices of order n <= G in one wave (G =
// 16: four, G = 32: two): the G-lane group q = lane / G inverts its own
// matrix, lane i of the group holding row i of [A | I] in registers.  Partial
// pivoting by the largest |entry| of the column among the rows not yet used as
// pivots (ties: the lowest row); the pivot row is scaled by the reciprocal of
// the pivot and broadcast through the group's LDS slot (2 G doubles), and every
// other row subtracts its multiple, the same arithmetic per entry as invert().
// The row that was the pivot of step k ends as row k of the inverse.  Aq /
// Aiq: the lane's group's input and output (row-major, may be the same
// buffer; Aq null: the group idles); slot: 128 doubles per wave.  Returns
// false on the lanes of a group whose matrix has a zero pivot column.
// (always inlined: a call left the caller's registers to the call ABI)
template <int G>
__device__ __forceinline__ bool invert_grp(int n, const double* Aq, double* Aiq, double* slot) {
    const int lane = (int)(threadIdx.x & 63), q = lane / G, i = lane % G;
    const bool grp = Aq != nullptr;
    const bool act = grp && i < n;
    double a[G], b[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
        a[j] = (act && j < n) ? Aq[i * n + j] : 0.0;
        b[j] = (act && i == j) ? 1.0 : 0.0;
    }
    double* sl = slot + q * 2 * G;
    bool used = false, ok = true;
    int stepk = -1;
    WaveTeam wt;
    wt.sync();  // every read of Aq precedes any write of Aiq
    // the step loop stays rolled: unrolled, the sixteen steps of G = 16 made
    // the finish kernel slower (measured 0.63 against 0.44 ms for 4096
    // elements); a[k] is picked by selects, not by a dynamic register index
#pragma unroll 1
    for (int k = 0; k < n; ++k) {
        double ak = 0.0;
#pragma unroll
        for (int j = 0; j < G; ++j)
            if (j == k) ak = a[j];
        double v = (act && !used) ? fabs(ak) : -1.0;
        int p = i;
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
            const double ov = __shfl_xor(v, off, G);
            const int op = __shfl_xor(p, off, G);
            if (ov > v || (ov == v && op < p)) {
                v = ov;
                p = op;
            }
        }
        const bool sing = !(v > 0.0);
        if (sing) ok = false;
        const bool piv = act && !sing && i == p;
        if (piv) {
            const double inv = 1.0 / ak;
#pragma unroll
            for (int j = 0; j < G; ++j) {
                a[j] *= inv;
                b[j] *= inv;
                sl[j] = a[j];
                sl[G + j] = b[j];
            }
            used = true;
            stepk = k;
        }
        wt.sync();
        if (act && !sing && !piv) {
            const double m = ak;
#pragma unroll
            for (int j = 0; j < G; ++j) {
                a[j] -= m * sl[j];
                b[j] -= m * sl[G + j];
            }
        }
        wt.sync();
    }
    if (act && stepk >= 0)
#pragma unroll
        for (int j = 0; j < G; ++j)
            if (j < n) Aiq[stepk * n + j] = b[j];
    wt.sync();
    return ok || !grp;
}
__device__ bool invert4(int n, const double* Aq, double* Aiq, double* slot) {
    return invert_grp<16>(n, Aq, Aiq, slot);
}

// Inverse of an upper quasi-triangular n x n matrix X (n <= G; a 2 x 2
// diagonal block wherever the subdiagonal entry is nonzero) by back
// substitution, one column per lane of the G-lane group: lane c solves
// X y = e_c from the last row up (a 2 x 2 block by Cramer's rule) with y in
// registers and X's rows read from LDS.  Xi (may alias X; every read of X
// precedes the first write) receives the inverse.  Returns false when a
// column is not finite (a singular diagonal block); null X: the group idles.
template <int G>
__device__ __forceinline__ bool qtri_inverse(int n, const double* X, double* Xi) {
    const int c = (int)(threadIdx.x % G);
    const bool act = X != nullptr && c < n;
    double y[G];
#pragma unroll
    for (int i = 0; i < G; ++i) y[i] = 0.0;
    bool below = false;  // row i + 1 closed a 2 x 2 block that solved row i too
#pragma unroll
    for (int i = G - 1; i >= 0; --i) {
        if (act && i < n) {
            if (below) {
                below = false;
            } else {
                double r = i == c ? 1.0 : 0.0;
#pragma unroll
                for (int k = i + 1; k < G; ++k)
                    if (k < n) r -= X[i * n + k] * y[k];
                const int i1 = i > 0 ? i - 1 : 0;  // the row above (i > 0 below)
                if (i > 0 && X[i * n + i1] != 0.0) {
                    double r1 = i1 == c ? 1.0 : 0.0;
#pragma unroll
                    for (int k = i + 1; k < G; ++k)
                        if (k < n) r1 -= X[i1 * n + k] * y[k];
                    const double a = X[i1 * n + i1], b = X[i1 * n + i];
                    const double d = X[i * n + i1], e = X[i * n + i];
                    const double det = a * e - b * d;
                    y[i1] = (r1 * e - b * r) / det;
                    y[i] = (a * r - d * r1) / det;
                    below = true;
                } else {
                    y[i] = r / X[i * n + i];
                }
            }
        }
    }
    double bad = 0.0;
#pragma unroll
    for (int k = 0; k < G; ++k)
        if (!(fabs(y[k]) < 1e300)) bad = 1.0;
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) bad = fmax(bad, __shfl_xor(bad, off, G));
    WaveTeam wt;
    wt.sync();  // every read of X precedes any write of Xi
    if (act)
#pragma unroll
        for (int k = 0; k < G; ++k)
            if (k < n) Xi[k * n + c] = y[k];
    wt.sync();
    return bad == 0.0 || X == nullptr;
}

// ||M||_1 (largest column sum of |entries|) of the lane's G-lane group's
// n x n matrix (n <= G), on every lane of the group
template <int G = 16>
__device__ double norm1_group(int n, const double* M) {
    const int i = (int)(threadIdx.x % G);
    double c = 0.0;
    if (M != nullptr && i < n)
        for (int r = 0; r < n; ++r) c += fabs(M[r * n + i]);
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) c = fmax(c, __shfl_xor(c, off, G));
    return c;
}

// Four-wave variants of prepare and finish (256 threads per element): the
// independent pieces of the work run on separate waves, each with its own
// LDS scratch, with the arithmetic of the one-wave kernels (the angle search
// compares the same scores with the same tie rule), except for the column
// inverses N_j.  The inversions run in registers, four at a time per wave
// for n <= 16 and two for n > 16: the factor inverses by invert_grp (the same
// operations per entry as invert(); its pivot order can differ only on exact
// ties), the N_j, whose inputs are upper quasi-triangular, by qtri_inverse
// (back substitution; equal to the one-wave kernel's Gauss-Jordan inverse
// to rounding).
//   prepare: wave w scores the rotation angles k = w and w + 4; the inverses
//            are formed by wave 0 (n <= 16) or waves 0..2; waves 0, 1 form
//            C1, C2.
//   finish:  waves 0, 1 form the two L = Q^T inverse tables; wave w forms
//            the N_j with j = w mod 4 (a 2 x 2 block of T2 stays on one wave).
template <bool kGrp4>
__global__ void __launch_bounds__(256) k_tables_prepare4(int64_t E, int dim, int n, int rank,
                                                         const double* factors, double* tab64,
                                                         int32_t* status, TabAddr ad) {
    extern __shared__ double lds[];
    __shared__ double red[4 * kMaxReduce];
    __shared__ double scores[8];
    __shared__ int fail[4];
    __shared__ double gslot[4][4 * 32];
    BlockTeam bt{red};
    WaveTeam wt;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long nn = (long)n * n;
    const int nf = dim == 2 ? 2 * rank : 5;
    // n <= 16: four matrices per wave are inverted at once (invert4), else two
    constexpr bool grp4 = kGrp4;
    const int wsz = grp4 ? 4 : 2;          // scratch matrices per wave
    double* F = lds;                       // nf n^2
    double* R6 = F + nf * nn;              // left 1
    double* R7 = R6 + nn;                  // left 2 (inverted)
    double* R8 = R7 + nn;                  // right 1 (inverted)
    double* R9 = R8 + nn;                  // right 2
    double* Wv = R9 + nn + wv * wsz * nn;  // this wave's scratch
    for (int64_t it = blockIdx.x; it < E; it += gridDim.x) {
        const int64_t e = ad.elem(it);
        for (long t = threadIdx.x; t < nf * nn; t += blockDim.x) F[t] = factors[ad.fac(e) + t];
        if (threadIdx.x < 4) fail[threadIdx.x] = 0;
        __syncthreads();
        double* tab = tab64 + ad.tab(e);
        double* N = tab + 7 * nn;
        for (long t = threadIdx.x; t < 3 * nn; t += blockDim.x) tab[t] = 0.0;
        // balance the norms within each term
        const double* l1 = dim == 2 ? F : F + nn;
        const double* l2 = dim == 2 ? F + 2 * nn : F + 3 * nn;
        const double* r1 = dim == 2 ? F + nn : F + 2 * nn;
        const double* r2 = dim == 2 ? F + 3 * nn : F + 4 * nn;
        double p1 = 0.0, p2 = 0.0;
        for (long t = threadIdx.x; t < nn; t += blockDim.x) {
            p1 += l1[t] * l1[t];
            p2 += l2[t] * l2[t];
        }
        const double s1 = sqrt(bt.sum(p1)), s2 = sqrt(bt.sum(p2));
        const double a1 = s1 > 0.0 ? s1 : 1.0, a2 = s2 > 0.0 ? s2 : 1.0;
        for (long t = threadIdx.x; t < nn; t += blockDim.x) {
            R6[t] = l1[t] / a1;
            R9[t] = r1[t] * a1;  // temporarily: balanced right 1
            R7[t] = l2[t] / a2;
            R8[t] = r2[t] * a2;  // temporarily: balanced right 2
        }
        __syncthreads();
        // angle search: kappa_1 of the two factors to invert for k = wv, wv + 4
        const double pi = 3.14159265358979323846;
        if (grp4) {
            // group 2h + m: angle wv + 4h, matrix m (0: rotated left 2, 1: rotated right 1)
            for (int h = 0; h < 2; ++h) {
                const int k = wv + 4 * h;
                const double c = cos(pi * k / 8.0), sn = sin(pi * k / 8.0);
                double* M0 = Wv + (2 * h) * nn;
                double* M1 = M0 + nn;
                for (long t = lane; t < nn; t += 64) {
                    M0[t] = -sn * R6[t] + c * R7[t];
                    M1[t] = c * R9[t] + sn * R8[t];
                }
            }
            wt.sync();
            double* Mq = Wv + (lane >> 4) * nn;
            const double nm = norm1_group(n, Mq);
            const bool ok = invert4(n, Mq, Mq, gslot[wv]);
            const double ni = norm1_group(n, Mq);
            const double term = ok ? nm * ni : 1e300;
            const double t0 = __shfl(term, 0, 64), t1 = __shfl(term, 16, 64);
            const double t2 = __shfl(term, 32, 64), t3 = __shfl(term, 48, 64);
            double sc0 = 1.0 * t0 * t1, sc1 = 1.0 * t2 * t3;
            if (!(sc0 == sc0)) sc0 = 1e300;
            if (!(sc1 == sc1)) sc1 = 1e300;
            if (lane == 0) {
                scores[wv] = sc0;
                scores[wv + 4] = sc1;
            }
            wt.sync();
        }
        for (int k = wv; k < 8 && !grp4; k += 4) {
            // 32-lane group m inverts matrix m (0: rotated left 2, 1: rotated right 1)
            const double c = cos(pi * k / 8.0), sn = sin(pi * k / 8.0);
            double* W0 = Wv;
            double* W1 = Wv + nn;
            for (long t = lane; t < nn; t += 64) {
                W0[t] = -sn * R6[t] + c * R7[t];
                W1[t] = c * R9[t] + sn * R8[t];
            }
            wt.sync();
            double* Mq = Wv + (lane >> 5) * nn;
            const double nm = norm1_group<32>(n, Mq);
            const bool ok = invert_grp<32>(n, Mq, Mq, gslot[wv]);
            const double ni = norm1_group<32>(n, Mq);
            const double term = ok ? nm * ni : 1e300;
            const double t0 = __shfl(term, 0, 64), t1 = __shfl(term, 32, 64);
            double score = 1.0 * t0 * t1;
            if (!(score == score)) score = 1e300;
            if (lane == 0) scores[k] = score;
            wt.sync();
        }
        __syncthreads();
        int bestk = 0;
        for (int k = 1; k < 8; ++k)
            if (scores[k] < scores[bestk]) bestk = k;
        {
            const double c = cos(pi * bestk / 8.0), sn = sin(pi * bestk / 8.0);
            for (long t = threadIdx.x; t < nn; t += blockDim.x) {
                const double bl1 = R6[t], bl2 = R7[t], br1 = R9[t], br2 = R8[t];
                R6[t] = c * bl1 + sn * bl2;
                R7[t] = -sn * bl1 + c * bl2;
                R8[t] = c * br1 + sn * br2;
                R9[t] = -sn * br1 + c * br2;
            }
        }
        __syncthreads();
        // inverses into the L slots: 2D L0 = inv(A2'), L1 = inv(B1');
        // 3D L0 = inv(A1), L1 = inv(B2'), L2 = inv(C1')
        const double* srcs[3] = {dim == 2 ? R7 : F, dim == 2 ? R8 : R7, R8};
        const int nq = dim == 3 ? 3 : 2;
        if (grp4 && wv == 0) {
            // wave 0 inverts all of them, group q the q-th, in its scratch
            for (int q = 0; q < nq; ++q)
                for (long t = lane; t < nn; t += 64) Wv[q * nn + t] = srcs[q][t];
            wt.sync();
            const int q = lane >> 4;
            double* Mq = q < nq ? Wv + q * nn : nullptr;
            const bool ok = invert4(n, Mq, Mq, gslot[0]);
            if (!ok && (lane & 15) == 0) fail[q] = 1;
            for (int qq = 0; qq < nq; ++qq)
                for (long t = lane; t < nn; t += 64) tab[qq * nn + t] = Wv[qq * nn + t];
            wt.sync();
        }
        if (!grp4 && wv < nq) {
            // wave q inverts the q-th in place (its lanes 32..63 idle)
            double* W0 = Wv;
            for (long t = lane; t < nn; t += 64) W0[t] = srcs[wv][t];
            wt.sync();
            if (!invert_grp<32>(n, lane < 32 ? W0 : nullptr, W0, gslot[wv]) && lane == 0) fail[wv] = 1;
            double* dst = tab + wv * nn;
            for (long t = lane; t < nn; t += 64) dst[t] = W0[t];
            wt.sync();
        }
        __syncthreads();
        // C1 = inv(Y) G_y, C2 = inv(Z) G_z (2D: Y = A2', Z = B1'; 3D: Y = B2', Z = C1')
        if (wv < 2) {
            const int src_wave = dim == 2 ? wv : wv + 1;  // the wave (grp4: wave 0's group) holding inv(Y) / inv(Z)
            const double* inv = grp4 ? lds + nf * nn + 4 * nn + src_wave * nn
                                     : lds + nf * nn + 4 * nn + src_wave * wsz * nn;
            const double* G = wv == 0 ? R6 : R9;
            double* out = grp4 ? Wv + 3 * nn : Wv + nn;  // clear of every inverse
            mm(wt, n, inv, G, out);
            for (long t = lane; t < nn; t += 64) N[wv * nn + t] = out[t];
            wt.sync();
        }
        __syncthreads();
        if (threadIdx.x == 0) status[e] |= (fail[0] | fail[1] | fail[2]) ? 2 : 0;
        __syncthreads();
    }
}

template <bool kGrp4>
__global__ void __launch_bounds__(256) k_tables_finish4(int64_t E, int dim, int n, double* tab64,
                                                        int8_t* kinds, int32_t* status, TabAddr ad) {
    extern __shared__ double lds[];
    __shared__ double red[4 * kMaxReduce];
    __shared__ int fail[4];
    __shared__ double gslot[4][4 * 32];
    BlockTeam bt{red};
    WaveTeam wt;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long nn = (long)n * n;
    constexpr bool grp4 = kGrp4;  // n <= 16: the wave's four N_j inverted at once (invert4)
    double* T1 = lds;
    double* Wv = lds + nn + wv * (grp4 ? 5 : 3) * nn;  // grp4: 4 inputs, M; else W0, W1, W4
                                                       // (L tables), two inputs and M (N_j)
    for (int64_t it = blockIdx.x; it < E; it += gridDim.x) {
        const int64_t e = ad.elem(it);
        double* tab = tab64 + ad.tab(e);
        double* N = tab + 7 * nn;
        const double* T2 = tab + 6 * nn;
        int8_t* kd = kinds + e * kMaxN;
        if (threadIdx.x < 4) fail[threadIdx.x] = 0;
        for (long t = threadIdx.x; t < nn; t += blockDim.x) T1[t] = tab[5 * nn + t];
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            int k = 0;
            if (j > 0 && T2[j * n + j - 1] != 0.0) k = 2;
            if (j + 1 < n && T2[(j + 1) * n + j] != 0.0) k = 1;
            kd[j] = (int8_t)k;
        }
        __syncthreads();
        double* W0 = Wv;
        double* W1 = Wv + nn;
        double* W4 = Wv + 2 * nn;
        // L = Q^T inverse: 2D L0, L1; 3D L1, L2 (waves 0 and 1)
        if (wv < 2) {
            double* Lq = dim == 2 ? tab + wv * nn : tab + (wv + 1) * nn;
            const double* Rq = tab + (3 + wv) * nn;
            for (long t = lane; t < nn; t += 64) {
                W0[t] = Lq[t];
                W4[t] = Rq[t];
            }
            wt.sync();
            mtm(wt, n, W4, W0, W1);
            for (long t = lane; t < nn; t += 64) Lq[t] = W1[t];
            wt.sync();
        }
        // N_j, j = wv mod 4
        if (grp4) {
            // group q: j = wv + 4 q; the input is T1 + t_j I, or M^2 - q s I
            // for a 2 x 2 block (M = T1 + p I), inverted in place
            double* In = Wv;
            double* Mt = Wv + 4 * nn;
            for (int q = 0; q < 4; ++q) {
                const int j = wv + 4 * q;
                if (j >= n || kd[j] == 1) continue;
                double* X = In + q * nn;
                if (kd[j] == 0) {
                    const double tj = T2[j * n + j];
                    for (long t = lane; t < nn; t += 64) X[t] = T1[t] + ((t / n == t % n) ? tj : 0.0);
                } else {
                    const double p = T2[j * n + j], qv = T2[(j - 1) * n + j], sv = T2[j * n + j - 1];
                    for (long t = lane; t < nn; t += 64) Mt[t] = T1[t] + ((t / n == t % n) ? p : 0.0);
                    wt.sync();
                    mm(wt, n, Mt, Mt, X);
                    for (long t = lane; t < nn; t += 64) X[t] = X[t] - ((t / n == t % n) ? qv * sv : 0.0);
                }
                wt.sync();
            }
            const int q = lane >> 4, jq = wv + 4 * q;
            double* Xq = (jq < n && kd[jq] != 1) ? In + q * nn : nullptr;
            // upper quasi-triangular (T1's block structure): back substitution
            if (!qtri_inverse<16>(n, Xq, Xq) && (lane & 15) == 0) fail[wv] = 1;
            for (int qq = 0; qq < 4; ++qq) {
                const int j = wv + 4 * qq;
                if (j >= n || kd[j] == 1) continue;
                for (long t = lane; t < nn; t += 64) {
                    N[(long)j * nn + t] = In[qq * nn + t];
                    if (kd[j] == 2) N[(long)(j - 1) * nn + t] = In[qq * nn + t];
                }
            }
            wt.sync();
        }
        // n > 16: the same, two N_j at a time (j = wv + 8 h + 4 q for the
        // 32-lane group q); scratch: the two inputs and M
        for (int h = 0; !grp4 && wv + 8 * h < n; ++h) {
            double* Mt = Wv + 2 * nn;
            for (int q = 0; q < 2; ++q) {
                const int j = wv + 8 * h + 4 * q;
                if (j >= n || kd[j] == 1) continue;
                double* X = Wv + q * nn;
                if (kd[j] == 0) {
                    const double tj = T2[j * n + j];
                    for (long t = lane; t < nn; t += 64) X[t] = T1[t] + ((t / n == t % n) ? tj : 0.0);
                } else {
                    const double p = T2[j * n + j], qv = T2[(j - 1) * n + j], sv = T2[j * n + j - 1];
                    for (long t = lane; t < nn; t += 64) Mt[t] = T1[t] + ((t / n == t % n) ? p : 0.0);
                    wt.sync();
                    mm(wt, n, Mt, Mt, X);
                    for (long t = lane; t < nn; t += 64) X[t] = X[t] - ((t / n == t % n) ? qv * sv : 0.0);
                }
                wt.sync();
            }
            const int q = lane >> 5, jq = wv + 8 * h + 4 * q;
            double* Xq = (jq < n && kd[jq] != 1) ? Wv + q * nn : nullptr;
            if (!qtri_inverse<32>(n, Xq, Xq) && (lane & 31) == 0) fail[wv] = 1;
            for (int qq = 0; qq < 2; ++qq) {
                const int j = wv + 8 * h + 4 * qq;
                if (j >= n || kd[j] == 1) continue;
                for (long t = lane; t < nn; t += 64) {
                    N[(long)j * nn + t] = Wv[qq * nn + t];
                    if (kd[j] == 2) N[(long)(j - 1) * nn + t] = Wv[qq * nn + t];
                }
            }
            wt.sync();
        }
        __syncthreads();
        // non-finite check (a NaN fails the comparison)
        double bad = 0.0;
        for (long t = threadIdx.x; t < 7L * nn; t += blockDim.x)
            if (!(fabs(tab[t]) < 1e300)) bad = 1.0;
        for (long t = threadIdx.x; t < (long)n * nn; t += blockDim.x)
            if (!(fabs(N[t]) < 1e300)) bad = 1.0;
        bad = bt.max(bad);
        if (threadIdx.x == 0) status[e] |= ((fail[0] | fail[1] | fail[2] | fail[3]) ? 2 : 0) | (bad != 0.0 ? 8 : 0);
        __syncthreads();
    }
}

// work item w = 2 e + i: real Schur form of C_(i+1), held in N slot i, into
// the T_(i+1) and R_i slots
__global__ void __launch_bounds__(64) k_tables_schur(int64_t E, int n, double* tab64,
                                                     int32_t* status, TabAddr ad) {
    extern __shared__ double lds[];
    __shared__ double red[kMaxReduce];
    __shared__ double sh[kMaxN + 8];
    BlockTeam tm{red};
    const long nn = (long)n * n;
    double* H = lds;
    double* Q = lds + nn;
    for (int64_t w = blockIdx.x; w < 2 * E; w += gridDim.x) {
        const int64_t e = ad.elem(w >> 1);
        const int i = (int)(w & 1);
        double* tab = tab64 + ad.tab(e);
        const int st = tables_schur(tm, n, tab + (7 + i) * nn, tab + (5 + i) * nn,
                                    tab + (3 + i) * nn, H, Q, sh);
        if (threadIdx.x == 0 && st) atomicOr(&status[e], st);
        __syncthreads();
    }
}

// the same with four work items per wave, one per 16-lane team, each with
// its own LDS (H, Q, small scratch): the reflector loops span at most n
// lanes, so a whole wave per item left three quarters of it idle
__global__ void __launch_bounds__(64) k_tables_schur16(int64_t E, int n, double* tab64, int32_t* status,
                                                       TabAddr ad) {
    extern __shared__ double lds[];
    GroupTeam16 tm;
    const long nn = (long)n * n;
    const int gq = (int)(threadIdx.x >> 4);
    double* H = lds + gq * (2 * nn + kMaxN + 8);
    double* Q = H + nn;
    double* sh = Q + nn;
    for (int64_t w0 = (int64_t)blockIdx.x * 4; w0 < 2 * E; w0 += (int64_t)gridDim.x * 4) {
        const int64_t w = w0 + gq;
        if (w < 2 * E) {
            const int64_t e = ad.elem(w >> 1);
            const int i = (int)(w & 1);
            double* tab = tab64 + ad.tab(e);
            const int st = tables_schur(tm, n, tab + (7 + i) * nn, tab + (5 + i) * nn, tab + (3 + i) * nn, H, Q, sh);
            if (tm.leader() && st) atomicOr(&status[e], st);
        }
        tm.sync();
    }
}

__global__ void __launch_bounds__(64) k_tables_finish(int64_t E, int dim, int n, double* tab64,
                                                      int8_t* kinds, int32_t* status, TabAddr ad) {
    extern __shared__ double lds[];  // 6 n^2 work doubles
    __shared__ double red[kMaxReduce];
    __shared__ double sh[kMaxN + 8];
    __shared__ int ipiv[kMaxN];
    BlockTeam tm{red};
    const long nn = (long)n * n;
    for (int64_t it = blockIdx.x; it < E; it += gridDim.x) {
        const int64_t e = ad.elem(it);
        double* tab = tab64 + ad.tab(e);
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
template <typename T, typename TT, class Rnd, class Z = double>
// axes (3D, or NULL): the elements' split axes; the tensor is loaded and
// stored in the relabelled order (y,x,z or z,x,y) of its element
__global__ void __launch_bounds__(256) k_apply_generic(int64_t E, int dim, int n, int nrhs,
                                                       const TT* tabs, int64_t tab_stride,
                                                       const int8_t* kinds, const double* r,
                                                       Z* z, Rnd rnd, const int8_t* axes) {
    extern __shared__ double lds[];
    __shared__ double red[4 * kMaxReduce];
    BlockTeam tm{red};
    const long nd = dim == 2 ? n * n : n * n * n;
    T* X = (T*)lds;
    T* Y = X + nd;
    T* H = Y + nd;
    for (int64_t w = blockIdx.x; w < E * nrhs; w += gridDim.x) {
        const int64_t e = w / nrhs;
        const int ax = (axes && dim == 3) ? axes[e] : 0;
        if (ax == 0) {
            for (long t = threadIdx.x; t < nd; t += blockDim.x) X[t] = (T)r[w * nd + t];
        } else {
            // logical (a, b, c) at a*n^2 + b*n + c; natural address a*sa + b*sb + c*sc
            const int sa = ax == 1 ? n : 1, sb = n * n, sc = ax == 1 ? 1 : n;
            for (long t = threadIdx.x; t < nd; t += blockDim.x) {
                const int a = (int)(t / (n * n)), bb = (int)((t / n) % n), cc = (int)(t % n);
                X[t] = (T)r[w * nd + a * sa + bb * sb + cc * sc];
            }
        }
        __syncthreads();
        apply_tensor(tm, dim, n, tabs + e * tab_stride, kinds + e * kMaxN, X, Y, H, rnd);
        // streaming stores: z is read only by a later kernel
        if (ax == 0) {
            for (long t = threadIdx.x; t < nd; t += blockDim.x)
                __builtin_nontemporal_store((Z)X[t], &z[w * nd + t]);
        } else {
            const int sa = ax == 1 ? n : 1, sb = n * n, sc = ax == 1 ? 1 : n;
            for (long t = threadIdx.x; t < nd; t += blockDim.x) {
                const int a = (int)(t / (n * n)), bb = (int)((t / n) % n), cc = (int)(t % n);
                __builtin_nontemporal_store((Z)X[t], &z[w * nd + a * sa + bb * sb + cc * sc]);
            }
        }
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

// Stage-1 Gram matrices of explicit blocks, G_e = R(A_e) R(A_e)^T (m = n^2 <=
// 64 rows, s^2 columns, s = n in 2D and n^2 in 3D), one wave per element on
// the FP64 matrix cores: 16 x 16 output tiles (P, Q), Q >= P, of 16 x 16 x 4
// products over the columns; the lane (g, c) loads R[16 P + c][k0 + g] of
// each row tile once and feeds it to every tile of that row or column tile.
// Rows past m and columns past s^2 read a valid entry and feed zero.  Each
// block entry is read once (the rearrangement is applied in the addressing).
__global__ void __launch_bounds__(256) k_explicit_gram(int64_t E, int n, int s, const double* blocks, double* grams) {
    typedef double dx4 __attribute__((ext_vector_type(4)));
    const int m = n * n;
    const long N = (long)n * s, len = (long)s * s, nd2 = N * N;
    const int lane = (int)(threadIdx.x & 63), g = lane >> 4, c = lane & 15;
    const int mt = (m + 15) / 16;
    long roff[4];
    bool rok[4];
#pragma unroll
    for (int P = 0; P < 4; ++P) {
        const int p = 16 * P + c;
        rok[P] = p < m;
        const int pp = rok[P] ? p : 0;
        roff[P] = ((long)(pp / n) * s) * N + (long)(pp % n) * s;
    }
    for (int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); e < E; e += (int64_t)gridDim.x * 4) {
        const double* A = blocks + e * nd2;
        dx4 acc[10];
#pragma unroll
        for (int t = 0; t < 10; ++t) acc[t] = dx4{0.0, 0.0, 0.0, 0.0};
        for (long k0 = 0; k0 < len; k0 += 8) {
            double r[2][4];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const long k = k0 + 4 * u + g;
                const bool kok = k < len;
                const long kk = kok ? k : len - 1;
                const long col = (kk / s) * N + kk % s;
#pragma unroll
                for (int P = 0; P < 4; ++P) {
                    const double v = A[roff[P] + col];
                    r[u][P] = (kok && rok[P]) ? v : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                int t = 0;
#pragma unroll
                for (int P = 0; P < 4; ++P)
#pragma unroll
                    for (int Q = P; Q < 4; ++Q, ++t)
                        if (Q < mt) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(r[u][P], r[u][Q], acc[t], 0, 0, 0);
            }
        }
        // the lane holds D[g + 4 v][c] of each tile
        double* G = grams + e * (long)m * m;
        int t = 0;
#pragma unroll
        for (int P = 0; P < 4; ++P)
#pragma unroll
            for (int Q = P; Q < 4; ++Q, ++t)
                if (Q < mt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = 16 * P + g + 4 * v, j = 16 * Q + c;
                        if (i < m && j < m) {
                            G[(long)i * m + j] = acc[t][v];
                            G[(long)j * m + i] = acc[t][v];
                        }
                    }
    }
}

hipError_t launch_explicit_gram(hipStream_t s, int64_t E, int dim, int n, const double* blocks, double* grams) {
    if (E <= 0) return hipSuccess;
    if (n * n > 64) return hipErrorInvalidValue;
    const int64_t wg = (E + 3) / 4;
    const int grid = (int)(wg < 65536 ? wg : 65536);
    hipLaunchKernelGGL(k_explicit_gram, dim3(grid), dim3(256), 0, s, E, n, dim == 3 ? n * n : n, blocks, grams);
    return hipGetLastError();
}

hipError_t launch_setup(hipStream_t s, int grid, int64_t E, int dim, int n, int rank,
                        const Tables1D* tab, const double* params, const double* blocks,
                        const double* guess, double* factors, double* sigma, int32_t* status,
                        double* ws, int64_t ws_stride, const int32_t* skip, int32_t status_or,
                        const double* grams) {
    const size_t small = setup_small_doubles(n, blocks != nullptr);
    if (rank >= 3) {
        hipLaunchKernelGGL(k_setup<true>, dim3(grid), dim3(256), small * sizeof(double), s, E, dim, n, rank,
                           tab, params, blocks, guess, factors, sigma, status, ws, ws_stride, skip, status_or,
                           grams);
    } else if (4 * ((small + 31) / 32 * 32) * sizeof(double) + sizeof(Tables1D) > kSetupWavesLdsMax) {
        // the four waves' small arrays do not fit: one workgroup per element
        hipLaunchKernelGGL(k_setup<false>, dim3(grid), dim3(256), small * sizeof(double), s, E, dim, n, rank,
                           tab, params, blocks, guess, factors, sigma, status, ws, ws_stride, skip, status_or,
                           grams);
    } else {
        // one wave per element: the grid's workspace slots (a multiple of 4,
        // see setup_slots) serve grid / 4 workgroups
        const int64_t small_stride = (small + 31) / 32 * 32;
        const int g4 = grid / 4;
        auto kern = dim == 3 ? (blocks ? k_setup_waves<false, 3, true> : k_setup_waves<false, 3, false>)
                             : (blocks ? k_setup_waves<false, 2, true> : k_setup_waves<false, 2, false>);
        hipLaunchKernelGGL(kern, dim3(g4), dim3(256), 4 * small_stride * sizeof(double), s, E, dim, n, rank,
                           tab, params, blocks, guess, factors, sigma, status, ws, ws_stride, skip, status_or,
                           small_stride, grams);
    }
    return hipGetLastError();
}

static hipError_t form_tables(hipStream_t s, int64_t E, int dim, int n, int rank, const double* factors,
                              double* tab64, int8_t* kinds, int32_t* status, TabAddr ad) {
    if (E <= 0) return hipSuccess;
    const long nn = (long)n * n;
    const int nf = dim == 2 ? 2 * rank : 5;
    // at most (6 + 10) 32^2 doubles = 128 KiB of LDS (2D rank 3, n = 32)
    const size_t lds = (nf + 10) * nn * sizeof(double);
    const int grid = (int)(E < 65536 ? E : 65536);
    // four-wave kernels where their scratch fits in LDS, else one wave per element
    const size_t lds4p = (nf + 4 + (n <= 16 ? 16 : 8)) * nn * sizeof(double);
    const size_t lds4f = (n <= 16 ? 21 : 13) * nn * sizeof(double);
    // 2D rank 1 has no pair to rotate: the one-wave kernel
    if (lds4p <= kTables4LdsMax && !(dim == 2 && rank == 1))
        hipLaunchKernelGGL(n <= 16 ? k_tables_prepare4<true> : k_tables_prepare4<false>, dim3(grid), dim3(256),
                           lds4p, s, E, dim, n, rank, factors,
                           tab64, status, ad);
    else
        hipLaunchKernelGGL(k_tables_prepare, dim3(grid), dim3(64), lds, s, E, dim, n, rank, factors,
                           tab64, status, ad);
    const int64_t items = 2 * E;
    const size_t lds16 = 4 * (2 * nn + kMaxN + 8) * sizeof(double);
    if (lds16 <= 64 * 1024) {
        const int64_t wg = (items + 3) / 4;
        const int grid16 = (int)(wg < 65536 ? wg : 65536);
        hipLaunchKernelGGL(k_tables_schur16, dim3(grid16), dim3(64), lds16, s, E, n, tab64, status, ad);
    } else {
        const int grid2 = (int)(items < 65536 ? items : 65536);
        hipLaunchKernelGGL(k_tables_schur, dim3(grid2), dim3(64), 2 * nn * sizeof(double), s, E, n,
                           tab64, status, ad);
    }
    if (lds4f <= kTables4LdsMax)
        hipLaunchKernelGGL(n <= 16 ? k_tables_finish4<true> : k_tables_finish4<false>, dim3(grid), dim3(256),
                           lds4f, s, E, dim, n, tab64, kinds,
                           status, ad);
    else
        hipLaunchKernelGGL(k_tables_finish, dim3(grid), dim3(64), 6 * nn * sizeof(double), s, E, dim, n,
                           tab64, kinds, status, ad);
    return hipGetLastError();
}

hipError_t launch_form_tables(hipStream_t s, int64_t E, int dim, int n, int rank,
                              const double* factors, double* tab64, int8_t* kinds,
                              int32_t* status) {
    const long nn = (long)n * n;
    const TabAddr ad{nullptr, nullptr, (dim == 2 ? 2 * rank : 5) * nn, tab_entries(n)};
    return form_tables(s, E, dim, n, rank, factors, tab64, kinds, status, ad);
}

hipError_t launch_form_tables_list(hipStream_t s, int64_t count, const int32_t* list, const MixedElem* el,
                                   int dim, int n, const double* factors, double* tab64, int8_t* kinds,
                                   int32_t* status) {
    return form_tables(s, count, dim, n, 2, factors, tab64, kinds, status, TabAddr{list, el, 0, 0});
}

hipError_t launch_cast_tables(hipStream_t s, int64_t count, const double* t64, float* t32,
                              uint16_t* hi, uint16_t* lo, float* t2) {
    int grid = (int)((count + 255) / 256);
    if (grid > 65536) grid = 65536;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_cast_tables, dim3(grid), dim3(256), 0, s, count, t64, t32, hi, lo, t2);
    return hipGetLastError();
}

template <class Z>
static hipError_t apply_generic(hipStream_t s, int prec, int64_t E, int dim, int n, int nrhs, const void* tabs,
                                int64_t tab_stride, const int8_t* kinds, const double* r, Z* z,
                                const int8_t* axes) {
    const long nd = dim == 2 ? n * n : n * n * n;
    int64_t work = E * nrhs;
    int grid = (int)(work < 65536 ? work : 65536);
    if (prec == 0) {
        size_t lds = 4 * nd * sizeof(double);
        hipLaunchKernelGGL((k_apply_generic<double, double, RoundNone, Z>), dim3(grid), dim3(256), lds, s,
                           E, dim, n, nrhs, (const double*)tabs, tab_stride, kinds, r, z, RoundNone(), axes);
    } else if (prec == 1) {
        size_t lds = 4 * nd * sizeof(float);
        hipLaunchKernelGGL((k_apply_generic<float, float, RoundNone, Z>), dim3(grid), dim3(256), lds, s,
                           E, dim, n, nrhs, (const float*)tabs, tab_stride, kinds, r, z, RoundNone(), axes);
    } else if (prec == 2) {
        size_t lds = 4 * nd * sizeof(float);
        hipLaunchKernelGGL((k_apply_generic<float, uint16_t, RoundBf16, Z>), dim3(grid), dim3(256), lds,
                           s, E, dim, n, nrhs, (const uint16_t*)tabs, tab_stride, kinds, r, z,
                           RoundBf16(), axes);
    } else {
        size_t lds = 4 * nd * sizeof(float);
        hipLaunchKernelGGL((k_apply_generic<float, float, RoundBf16x2, Z>), dim3(grid), dim3(256), lds,
                           s, E, dim, n, nrhs, (const float*)tabs, tab_stride, kinds, r, z,
                           RoundBf16x2(), axes);
    }
    return hipGetLastError();
}

// ------------------------------------------- split-axis choice (3D records)
// out[k - 1][e] = record e with its axes relabelled so that axis k comes first
// (orders y,x,z and z,x,y): the per-axis data (beta, the two face velocities
// of each axis) permuted; the mass coefficient of the record,
// 1 + alpha sin(pi x y z + phi), is symmetric in the axes
__global__ void k_permute_records(int64_t E, const double* params, double* out) {
    const int64_t count = 2 * E;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < count;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(q / E) + 1;
        const int64_t e = q % E;
        const double* src = params + e * kRecLen;
        double* dst = out + q * kRecLen;
        const int o[3] = {k, 0, k == 1 ? 2 : 1};
        for (int i = 0; i < kRecLen; ++i) dst[i] = src[i];
        for (int a = 0; a < 3; ++a) {
            dst[a] = src[o[a]];
            dst[8 + 2 * a] = src[8 + 2 * o[a]];
            dst[9 + 2 * a] = src[9 + 2 * o[a]];
        }
    }
}

// per element, the axis whose stage-1 sigma_1 is largest (ties to the lowest);
// axis 0's results are in place (factors, sigma, status), axes 1 and 2 in
// fac[k - 1], sig[k - 1], st[k - 1]; the winner's are copied in place
__global__ void __launch_bounds__(256) k_choose_axis(int64_t E, int64_t nfnn, const double* fac, const double* sig,
                                                     const int32_t* st, double* factors, double* sigma,
                                                     int32_t* status, int8_t* axis) {
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const double s0 = sigma[e * 4], s1 = sig[e * 4], s2 = sig[(E + e) * 4];
        int k = 0;
        double best = s0;
        if (s1 > best) { best = s1; k = 1; }
        if (s2 > best) { best = s2; k = 2; }
        if (k != 0) {
            const int64_t base = (int64_t)(k - 1) * E + e;
            for (int64_t t = threadIdx.x; t < nfnn; t += blockDim.x) factors[e * nfnn + t] = fac[base * nfnn + t];
            if (threadIdx.x < 4) sigma[e * 4 + threadIdx.x] = sig[base * 4 + threadIdx.x];
            if (threadIdx.x == 0) status[e] = st[base];
        }
        if (threadIdx.x == 0) axis[e] = (int8_t)k;
    }
}

__global__ void k_fill_i8(int64_t count, int8_t* p, int8_t v) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x)
        p[q] = v;
}

hipError_t launch_permute_records(hipStream_t s, int64_t E, const double* params, double* out) {
    if (E <= 0) return hipSuccess;
    int64_t g = (2 * E + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_permute_records, dim3((int)g), dim3(256), 0, s, E, params, out);
    return hipGetLastError();
}

hipError_t launch_choose_axis(hipStream_t s, int64_t E, int64_t nfnn, const double* fac, const double* sig,
                              const int32_t* st, double* factors, double* sigma, int32_t* status, int8_t* axis) {
    if (E <= 0) return hipSuccess;
    const int grid = (int)(E < 65536 ? E : 65536);
    hipLaunchKernelGGL(k_choose_axis, dim3(grid), dim3(256), 0, s, E, nfnn, fac, sig, st, factors, sigma, status,
                       axis);
    return hipGetLastError();
}

hipError_t launch_fill_i8(hipStream_t s, int64_t count, int8_t* p, int8_t v) {
    if (count <= 0) return hipSuccess;
    int64_t g = (count + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_fill_i8, dim3((int)g), dim3(256), 0, s, count, p, v);
    return hipGetLastError();
}

hipError_t launch_apply_generic(hipStream_t s, int prec, int64_t E, int dim, int n, int nrhs,
                                const void* tabs, int64_t tab_stride, const int8_t* kinds,
                                const double* r, double* z, const int8_t* axes) {
    return apply_generic(s, prec, E, dim, n, nrhs, tabs, tab_stride, kinds, r, z, axes);
}

hipError_t launch_apply_generic(hipStream_t s, int prec, int64_t E, int dim, int n, int nrhs,
                                const void* tabs, int64_t tab_stride, const int8_t* kinds,
                                const double* r, float* z, const int8_t* axes) {
    if (prec == 0) return hipErrorInvalidValue;  // FP64 arithmetic: z stays FP64
    return apply_generic(s, prec, E, dim, n, nrhs, tabs, tab_stride, kinds, r, z, axes);
}

}  // namespace kp
