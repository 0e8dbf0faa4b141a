// Global operator and the vector kernels of FGMRES.
//
// The operator is the implicit system M - tau*J of the synthetic DG
// discretisation: each element's diagonal block (explicit, or matrix-free from
// its record) plus the upwind inflow coupling to the neighbour across every
// inflow face (Sec. 3.4.1, face part of eq. jac-entries).  With one normal
// velocity u_f per face (record entries 8..13, u_f > 0 outflow), an element takes the neighbour's trace on each inflow face f (u_f < 0): the
// coupling block is tau*u_f (l_f l_opp^T on the face's axis) times W on the
// other axes, l_f = l0 / l1 on the low / high face and l_opp the neighbour's
// opposite face.
#include <hip/hip_runtime.h>

#include "elem_ops.h"
#include "krylov.h"

namespace kp {

// One workgroup per element.  LDS: x_e, mass, X_ax, one face trace.  X: the
// type x is stored in (float for an FGMRES basis of FP32 preconditioner
// outputs; every value is taken to FP64 exactly on load).
template <class X>
__global__ void __launch_bounds__(256) k_operator(int64_t E, int dim, int n, const Tables1D* tab,
                                                  const double* params, const int32_t* nbr,
                                                  const double* blocks, const double* strc,
                                                  const X* x, double* y) {
    extern __shared__ double lds[];
    __shared__ double red[4 * kMaxReduce];
    __shared__ Tables1D T;
    BlockTeam tm{red};
    {
        const double* src = (const double*)tab;
        double* dst = (double*)&T;
        for (int i = threadIdx.x; i < (int)(sizeof(Tables1D) / sizeof(double)); i += blockDim.x)
            dst[i] = src[i];
        __syncthreads();
    }
    const int nn = n * n;
    const int nd = dim == 2 ? nn : nn * n;
    const int nf = nd / n;  // face size n^(d-1)
    // LDS: x of the element, the axis matrices, a face trace; the mass tensor
    // too when it is formed here (with strc each thread reads its own entries
    // of it from HBM, which keeps the LDS footprint and so the occupancy down)
    double* xe = lds;
    double* Xax = xe + nd;
    double* tr = Xax + 3 * nn;
    double* mass_l = tr + nf;
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const double* rec = params + e * kRecLen;
        for (int t = threadIdx.x; t < nd; t += blockDim.x) xe[t] = (double)x[e * nd + t];
        const double* mass;
        if (strc) {
            const double* se = strc + e * (int64_t)(nd + 3 * nn);
            for (int t = threadIdx.x; t < 3 * nn; t += blockDim.x) Xax[t] = se[nd + t];
            mass = se;
            __syncthreads();
        } else {
            record_structure(tm, rec, T, dim, mass_l, Xax);  // ends with a barrier
            mass = mass_l;
        }
        double acc[16];
        const int per = (nd + blockDim.x - 1) / blockDim.x;
        for (int q = 0; q < per && q < 16; ++q) {
            const int I = threadIdx.x + q * blockDim.x;
            double v = 0.0;
            if (I < nd) {
                if (blocks) {
                    const double* row = blocks + (e * nd + I) * (int64_t)nd;
                    #pragma unroll 8
                    for (int J = 0; J < nd; ++J) v += row[J] * xe[J];
                } else {
                    v = mass[I] * xe[I];
                    int idx[3];
                    if (dim == 2) { idx[0] = I / n; idx[1] = I % n; }
                    else { idx[0] = I / nn; idx[1] = (I / n) % n; idx[2] = I % n; }
                    for (int ax = 0; ax < dim; ++ax) {
                        int stride = 1;
                        for (int k = ax + 1; k < dim; ++k) stride *= n;
                        double wp = 1.0;
                        for (int k = 0; k < dim; ++k)
                            if (k != ax) wp *= T.w[idx[k]];
                        const double* Xr = Xax + ax * nn + idx[ax] * n;
                        const int base = I - idx[ax] * stride;
                        double s = 0.0;
                        #pragma unroll 8
                        for (int k = 0; k < n; ++k) s += Xr[k] * xe[base + k * stride];
                        v += wp * s;
                    }
                }
            }
            acc[q] = v;
        }
        // upwind coupling on inflow faces
        if (nbr && rec[7] != 0.0) {
            for (int f = 0; f < 2 * dim; ++f) {
                const double u = rec[8 + f];
                if (!(u < 0.0)) continue;  // uniform across the workgroup
                const int ax = f >> 1, side = f & 1;
                const double* l_in = side ? T.l1 : T.l0;
                const double* l_out = side ? T.l0 : T.l1;
                const int64_t nb = nbr[e * 2 * dim + f];
                int stride = 1;
                for (int k = ax + 1; k < dim; ++k) stride *= n;
                // neighbour's trace on its opposite face: tr[J] = sum_k l_out[k] x_nb[..k..]
                const X* xf = x + nb * nd;
                for (int J = threadIdx.x; J < nf; J += blockDim.x) {
                    const int lo = J % stride, hi = J / stride;
                    const int base = hi * stride * n + lo;
                    double s = 0.0;
                    #pragma unroll 8
                    for (int k = 0; k < n; ++k) s += l_out[k] * (double)xf[base + k * stride];
                    tr[J] = s;
                }
                __syncthreads();
                const double coef = rec[6] * u;
                for (int q = 0; q < per && q < 16; ++q) {
                    const int I = threadIdx.x + q * blockDim.x;
                    if (I >= nd) continue;
                    int idx[3];
                    if (dim == 2) { idx[0] = I / n; idx[1] = I % n; }
                    else { idx[0] = I / nn; idx[1] = (I / n) % n; idx[2] = I % n; }
                    double wp = 1.0;
                    for (int k = 0; k < dim; ++k)
                        if (k != ax) wp *= T.w[idx[k]];
                    const int lo = I % stride, hi = I / (stride * n);
                    acc[q] += coef * l_in[idx[ax]] * wp * tr[hi * stride + lo];
                }
                __syncthreads();
            }
        }
        for (int q = 0; q < per && q < 16; ++q) {
            const int I = threadIdx.x + q * blockDim.x;
            if (I < nd) y[e * nd + I] = acc[q];
        }
        __syncthreads();
    }
}

// The same operator for 3D elements with n <= 16 whose structure is cached
// (strc): thread (b, c) of an element holds the column x[., b, c] in
// registers and forms y[a, b, c] for every a; x of the element, X0, X1, X2
// (transposed) and the six face traces of the inflow neighbours sit in LDS
// (the traces are formed first, all loads of a trace in flight together).
// 256 / n^2 elements per workgroup.  Every entry is formed from the terms of
// k_operator in the same order (mass term, the three axes, then the inflow
// faces in face order); the two agree to rounding (the compiler may fuse
// multiply-adds differently).
template <class X>
__global__ void __launch_bounds__(256) k_operator3_cols(int64_t E, int n, const Tables1D* tab,
                                                        const double* params, const int32_t* nbr,
                                                        const double* strc, const X* x, double* y) {
    extern __shared__ double lds[];
    const int nn = n * n, nd = nn * n;
    const int epw = 256 / nn;                 // elements per workgroup
    const int slot = (int)threadIdx.x / nn;   // this thread's element slot
    const int bc = (int)threadIdx.x % nn, b = bc / n, c = bc % n;
    const bool act = slot < epw;
    double* xs = lds + (act ? slot : 0) * (nd + 9 * nn);  // x of the element (n^3)
    double* X0 = xs + nd;                                 // axis-0 matrix
    double* X1 = X0 + nn;                                 // axis-1 matrix
    double* X2t = X1 + nn;                                // axis-2 matrix, transposed
    double* trs = X2t + nn;                               // face f's trace at trs + f n^2
    const double* w = tab->w;
    const double wb = act ? w[b] : 0.0, wc = act ? w[c] : 0.0;
    for (int64_t e0 = (int64_t)blockIdx.x * epw; e0 < E; e0 += (int64_t)gridDim.x * epw) {
        const int64_t e = e0 + slot;
        const bool live = act && e < E;
        const double* se = strc + (live ? e : 0) * (int64_t)(nd + 3 * nn);
        const double* rec = params + (live ? e : 0) * kRecLen;
        const bool faces = live && nbr && rec[7] != 0.0;
        double xc[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) xc[k] = (live && k < n) ? (double)x[e * nd + k * nn + bc] : 0.0;
        if (live) {
            X0[bc] = se[nd + bc];
            X1[bc] = se[nd + nn + bc];
            X2t[c * n + b] = se[nd + 2 * nn + bc];  // X2[b][c] at (c, b)
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (k < n) xs[k * nn + bc] = xc[k];
        }
        // the inflow faces' traces of the neighbours: face f's entry at
        // (b, c) is, for axis 0, the trace at (b, c); axis 1, at (a, c) = (b, c);
        // axis 2, at (a, b) = (b, c)
        for (int f = 0; f < 6; ++f) {
            if (!(faces && rec[8 + f] < 0.0)) continue;
            const int ax = f >> 1;
            const double* l_out = (f & 1) ? tab->l0 : tab->l1;
            const X* xf = x + (int64_t)nbr[e * 6 + f] * nd;
            double xv[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int J = ax == 0 ? k * nn + bc : ax == 1 ? b * nn + k * n + c : b * nn + c * n + k;
                xv[k] = k < n ? (double)xf[J] : 0.0;
            }
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (k < n) sum += l_out[k] * xv[k];
            trs[f * nn + bc] = sum;
        }
        __syncthreads();
        if (live) {
            // the mass column first, its loads in flight together
            double mv[16];
#pragma unroll
            for (int a = 0; a < 16; ++a) mv[a] = a < n ? se[a * nn + bc] : 0.0;
#pragma unroll
            for (int a = 0; a < 16; ++a) {
                if (a >= n) break;
                const int I = a * nn + bc;
                double v = mv[a] * xs[I];
                // axis 0: w_b w_c sum_k X0[a][k] x[k, b, c]
                {
                    const double wp = 1.0 * wb * wc;
                    double sum = 0.0;
#pragma unroll
                    for (int k = 0; k < 16; ++k)
                        if (k < n) sum += X0[a * n + k] * xc[k];
                    v += wp * sum;
                }
                const double wa = w[a];
                // axis 1: w_a w_c sum_k X1[b][k] x[a, k, c]
                {
                    const double wp = 1.0 * wa * wc;
                    double sum = 0.0;
#pragma unroll
                    for (int k = 0; k < 16; ++k)
                        if (k < n) sum += X1[b * n + k] * xs[a * nn + k * n + c];
                    v += wp * sum;
                }
                // axis 2: w_a w_b sum_k X2[c][k] x[a, b, k]
                {
                    const double wp = 1.0 * wa * wb;
                    double sum = 0.0;
#pragma unroll
                    for (int k = 0; k < 16; ++k)
                        if (k < n) sum += X2t[k * n + c] * xs[a * nn + b * n + k];
                    v += wp * sum;
                }
                // upwind coupling on the inflow faces, in face order
                if (faces) {
                    for (int f = 0; f < 6; ++f) {
                        const double u = rec[8 + f];
                        if (!(u < 0.0)) continue;
                        const int ax = f >> 1;
                        const double* l_in = (f & 1) ? tab->l1 : tab->l0;
                        const double coef = rec[6] * u;
                        const double* tf = trs + f * nn;
                        double wp, li, tr;
                        if (ax == 0) { wp = 1.0 * wb * wc; li = l_in[a]; tr = tf[bc]; }
                        else if (ax == 1) { wp = 1.0 * wa * wc; li = l_in[b]; tr = tf[a * n + c]; }
                        else { wp = 1.0 * wa * wb; li = l_in[c]; tr = tf[a * n + b]; }
                        v += coef * li * wp * tr;
                    }
                }
                y[e * nd + I] = v;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------- vector kernels
// partial[b * k + i] = sum over block b's entries of V_i . w   (i < k), the
// blocks striding over the vector.  Eight V_i per pass, so w is read
// ceil(k / 8) times; PAIR: two entries per thread and load (16 bytes; N and
// the vector stride even, the vectors 16-byte aligned), which keeps more bytes
// in flight per wave.
template <bool PAIR>
__global__ void __launch_bounds__(256) k_mdot_partial(const double* V, int64_t ldv, int k,
                                                      const double* w, int64_t N, double* partial) {
    constexpr int kG = 8;
    __shared__ double red[kG][4];
    const int nw = blockDim.x >> 6, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t M = PAIR ? N / 2 : N;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int i0 = 0; i0 < k; i0 += kG) {
        const int kk = k - i0 < kG ? k - i0 : kG;
        const double* v = V + i0 * ldv;
        double s[kG];
#pragma unroll
        for (int q = 0; q < kG; ++q) s[q] = 0.0;
        for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < M; t += stride) {
            if (PAIR) {
                const double2 wt = ((const double2*)w)[t];
#pragma unroll
                for (int q = 0; q < kG; ++q)
                    if (q < kk) {
                        const double2 x = ((const double2*)(v + q * ldv))[t];
                        s[q] += x.x * wt.x;
                        s[q] += x.y * wt.y;
                    }
            } else {
                const double wt = w[t];
#pragma unroll
                for (int q = 0; q < kG; ++q)
                    if (q < kk) s[q] += v[q * ldv + t] * wt;
            }
        }
        if (PAIR && (N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
            const double wt = w[N - 1];
#pragma unroll
            for (int q = 0; q < kG; ++q)
                if (q < kk) s[q] += v[q * ldv + N - 1] * wt;
        }
#pragma unroll
        for (int q = 0; q < kG; ++q)
            if (q < kk) {
                const double r = wave_sum(s[q]);
                if (lane == 0) red[q][wv] = r;
            }
        __syncthreads();
        if (threadIdx.x < kk) {
            double a = 0.0;
            for (int q = 0; q < nw; ++q) a += red[threadIdx.x][q];
            partial[blockIdx.x * (int64_t)k + i0 + threadIdx.x] = a;
        }
        __syncthreads();
    }
}

// out[i] = sum_b partial[b * k + i] (fixed order), optionally accumulated
// one workgroup per output: thread t sums the partials b = t, t + 256, ... in
// order, then a fixed-order reduction over the workgroup (deterministic)
__global__ void __launch_bounds__(256) k_mdot_reduce(const double* partial, int nblocks, int k, double* out,
                                                     int accumulate) {
    __shared__ double red[4];
    const int i = blockIdx.x;
    double a = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) a += partial[(int64_t)b * k + i];
    a = wave_sum(a);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        out[i] = accumulate ? out[i] + t : t;
    }
}

// w -= sum_i h[i] V_i (PAIR as for k_mdot_partial, the last entry of an odd N
// by thread 0 of block 0)
template <bool PAIR>
__global__ void k_mgs_update(const double* V, int64_t ldv, int k, const double* h, double* w,
                             int64_t N) {
    const int64_t M = PAIR ? N / 2 : N;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < M;
         t += (int64_t)gridDim.x * blockDim.x) {
        if (PAIR) {
            double2 s = ((const double2*)w)[t];
            for (int i = 0; i < k; ++i) {
                const double2 v = ((const double2*)(V + i * ldv))[t];
                const double hi = h[i];
                s.x -= hi * v.x;
                s.y -= hi * v.y;
            }
            ((double2*)w)[t] = s;
        } else {
            double s = w[t];
            for (int i = 0; i < k; ++i) s -= h[i] * V[i * ldv + t];
            w[t] = s;
        }
    }
    if (PAIR && (N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        double s = w[N - 1];
        for (int i = 0; i < k; ++i) s -= h[i] * V[i * ldv + N - 1];
        w[N - 1] = s;
    }
}

// x += sum_i y[i] Z_i (Z FP64 or FP32, taken to FP64 exactly)
template <class ZT>
__global__ void k_combine(const ZT* Z, int64_t ldz, int k, const double* y, double* x, int64_t N) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < N;
         t += (int64_t)gridDim.x * blockDim.x) {
        double s = x[t];
        for (int i = 0; i < k; ++i) s += y[i] * (double)Z[i * ldz + t];
        x[t] = s;
    }
}

// dst = a * src + b * other  (other may be null)
__global__ void k_axpby(double* dst, const double* src, double a, const double* other, double b,
                        int64_t N) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < N;
         t += (int64_t)gridDim.x * blockDim.x)
        dst[t] = a * src[t] + (other ? b * other[t] : 0.0);
}

// vn = w / sqrt(max(nrm2[0], 0)) (the same arithmetic as k_axpby with
// a = 1 / sqrt(...) computed on the host); zeros where the norm is zero
__global__ void k_normalize(const double* nrm2, const double* w, double* vn, int64_t N) {
    const double hn = sqrt(fmax(nrm2[0], 0.0));
    const double a = hn > 0.0 ? 1.0 / hn : 0.0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < N;
         t += (int64_t)gridDim.x * blockDim.x)
        vn[t] = a * w[t] + 0.0;
}

// ------------------------------------------------------------ launchers
template <class X>
static hipError_t operator_any(hipStream_t s, int64_t E, int dim, int n, const Tables1D* tab,
                               const double* params, const int32_t* nbr, const double* blocks,
                               const double* strc, const X* x, double* y, bool cols) {
    const int nn = n * n;
    const int nd = dim == 2 ? nn : nn * n;
    if (nd > 16 * 256) return hipErrorInvalidValue;
    const double* sc = blocks ? nullptr : strc;
    if (cols && sc && dim == 3 && n <= 16) {
        const int epw = 256 / nn;
        const int64_t wg = (E + epw - 1) / epw;
        const int grid3 = (int)(wg < 65536 ? wg : 65536);
        const size_t lds3 = (size_t)epw * (nd + 9 * nn) * sizeof(double);
        hipLaunchKernelGGL(k_operator3_cols<X>, dim3(grid3), dim3(256), lds3, s, E, n, tab, params, nbr, sc, x, y);
        return hipGetLastError();
    }
    size_t lds = ((sc ? 1 : 2) * nd + 3 * nn + nd / n) * sizeof(double);
    int grid = (int)(E < 65536 ? E : 65536);
    hipLaunchKernelGGL(k_operator<X>, dim3(grid), dim3(256), lds, s, E, dim, n, tab, params, nbr, blocks,
                       sc, x, y);
    return hipGetLastError();
}

hipError_t launch_operator(hipStream_t s, int64_t E, int dim, int n, const Tables1D* tab,
                           const double* params, const int32_t* nbr, const double* blocks,
                           const double* strc, const double* x, double* y, bool cols) {
    return operator_any(s, E, dim, n, tab, params, nbr, blocks, strc, x, y, cols);
}

hipError_t launch_operator(hipStream_t s, int64_t E, int dim, int n, const Tables1D* tab,
                           const double* params, const int32_t* nbr, const double* blocks,
                           const double* strc, const float* x, double* y, bool cols) {
    return operator_any(s, E, dim, n, tab, params, nbr, blocks, strc, x, y, cols);
}

// the matrix-free elements' structure: per element the mass tensor (n^d) and
// the three axis matrices (3 n^2) of record_structure, contiguous
__global__ void __launch_bounds__(256) k_structure(int64_t E, int dim, int n, const Tables1D* tab,
                                                   const double* params, double* strc) {
    __shared__ double red[4 * kMaxReduce];
    __shared__ Tables1D T;
    BlockTeam tm{red};
    {
        const double* src = (const double*)tab;
        double* dst = (double*)&T;
        for (int i = threadIdx.x; i < (int)(sizeof(Tables1D) / sizeof(double)); i += blockDim.x)
            dst[i] = src[i];
        __syncthreads();
    }
    const int nn = n * n;
    const int nd = dim == 2 ? nn : nn * n;
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        double* se = strc + e * (int64_t)(nd + 3 * nn);
        record_structure(tm, params + e * kRecLen, T, dim, se, se + nd);
    }
}

hipError_t launch_structure(hipStream_t s, int64_t E, int dim, int n, const Tables1D* tab,
                            const double* params, double* strc) {
    if (E <= 0) return hipSuccess;
    const int grid = (int)(E < 65536 ? E : 65536);
    hipLaunchKernelGGL(k_structure, dim3(grid), dim3(256), 0, s, E, dim, n, tab, params, strc);
    return hipGetLastError();
}

int vec_grid(int64_t N) {
    int64_t g = (N + 255) / 256;
    if (g > kVecBlocks) g = kVecBlocks;
    if (g < 1) g = 1;
    return (int)g;
}

// two entries per thread and 16-byte loads where every vector allows them
static bool pairs_ok(const double* V, int64_t ldv, int k, const double* w, int64_t N) {
    return N >= 2 && (k <= 1 || ldv % 2 == 0) && ((uintptr_t)V % 16) == 0 && ((uintptr_t)w % 16) == 0;
}

hipError_t launch_mdot(hipStream_t s, const double* V, int64_t ldv, int k, const double* w,
                       int64_t N, double* partial, double* out, int accumulate) {
    const int g = vec_grid(N);
    if (pairs_ok(V, ldv, k, w, N))
        hipLaunchKernelGGL(k_mdot_partial<true>, dim3(g), dim3(256), 0, s, V, ldv, k, w, N, partial);
    else
        hipLaunchKernelGGL(k_mdot_partial<false>, dim3(g), dim3(256), 0, s, V, ldv, k, w, N, partial);
    if (k > 0)
        hipLaunchKernelGGL(k_mdot_reduce, dim3(k), dim3(256), 0, s, partial, g, k, out, accumulate);
    return hipGetLastError();
}

hipError_t launch_mgs_update(hipStream_t s, const double* V, int64_t ldv, int k, const double* h,
                             double* w, int64_t N) {
    if (pairs_ok(V, ldv, k, w, N))
        hipLaunchKernelGGL(k_mgs_update<true>, dim3(vec_grid(N)), dim3(256), 0, s, V, ldv, k, h, w, N);
    else
        hipLaunchKernelGGL(k_mgs_update<false>, dim3(vec_grid(N)), dim3(256), 0, s, V, ldv, k, h, w, N);
    return hipGetLastError();
}

hipError_t launch_combine(hipStream_t s, const double* Z, int64_t ldz, int k, const double* y,
                          double* x, int64_t N) {
    hipLaunchKernelGGL(k_combine<double>, dim3(vec_grid(N)), dim3(256), 0, s, Z, ldz, k, y, x, N);
    return hipGetLastError();
}

hipError_t launch_combine(hipStream_t s, const float* Z, int64_t ldz, int k, const double* y,
                          double* x, int64_t N) {
    hipLaunchKernelGGL(k_combine<float>, dim3(vec_grid(N)), dim3(256), 0, s, Z, ldz, k, y, x, N);
    return hipGetLastError();
}

hipError_t launch_axpby(hipStream_t s, double* dst, const double* src, double a, const double* other,
                        double b, int64_t N) {
    hipLaunchKernelGGL(k_axpby, dim3(vec_grid(N)), dim3(256), 0, s, dst, src, a, other, b, N);
    return hipGetLastError();
}

hipError_t launch_normalize(hipStream_t s, const double* nrm2, const double* w, double* vn, int64_t N) {
    hipLaunchKernelGGL(k_normalize, dim3(vec_grid(N)), dim3(256), 0, s, nrm2, w, vn, N);
    return hipGetLastError();
}

}  // namespace kp
