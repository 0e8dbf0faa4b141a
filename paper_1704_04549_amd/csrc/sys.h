// Blocks of nc-component systems (2D): KSVD with nc n x nc n first factors
// (the component index grouped with x; Sec. 5.3), the inversion data and the
// apply of the Kronecker-sum inverse.
//
// Nodal vectors are ordered (component, x, y), component slowest; the block
// is explicit, (m n) x (m n) row-major with m = nc n.  Its rearrangement R(A)
// is m^2 x n^2 (rows: pairs of (component, x) indices; columns: pairs of y
// indices).  Setup: Lanczos (Alg. 2) on the smaller Gram R^T R, then
// A_j = sqrt(sigma_j) u_j (m x m), B_j = sqrt(sigma_j) v_j (n x n).
// Inversion data (Alg. 5): C1 = A2^-1 A1 (m x m), C2 = B1^-1 B2 (n x n), real
// Schur forms C1 = QA TA QA^T, C2 = QB TB QB^T, LA = QA^T A2^-1,
// LB = QB^T B1^-1, and the column inverses of the quasi-triangular Sylvester
// sweep over the n columns of TB: N_j = (TA + t_jj I)^-1 (m x m) for a real
// eigenvalue t_jj; for a 2 x 2 block of TB the real and imaginary parts of one
// complex inverse (TA + (p - i w) I)^-1 (see tables_sys).
// Apply: X (m x n) -> LA X LB^T -> Sylvester TA Y + Y TB^T = F -> QA Y QB^T.
#pragma once

#include "elem_ops.h"
#include "tables.h"

namespace kp {

constexpr int kSysMaxM = kMaxN;  // nc n <= 32

// entries of one element's apply tables: LA, LB, QA, QB, TA, TB, N_0..N_{n-1}
KP_INLINE long sys_tab_entries(int m, int n) {
    return 3L * m * m + 3L * n * n + (long)n * m * m;
}
struct SysTab {
    long LA, LB, QA, QB, TA, TB, N;
};
KP_INLINE SysTab sys_tab(int m, int n) {
    const long mm = (long)m * m, nn = (long)n * n;
    return SysTab{0, mm, mm + nn, 2 * mm + nn, 2 * mm + 2 * nn, 3 * mm + 2 * nn, 3 * mm + 3 * nn};
}
// factor stack of one element: A1 (m^2), B1 (n^2), A2 (m^2), B2 (n^2)
KP_INLINE long sys_factor_entries(int m, int n) { return 2L * m * m + 2L * n * n; }

// Lanczos runs on the right (y-pair) space, whose dimension n^2 is the smaller
// one: R^T R (n^2 x n^2) is formed once from the block and held in the
// workspace, and every left vector is recovered as R v.
// Preconditioner buffer of E system elements, structure of arrays, every
// section 256-byte aligned: factors [E][A1 m^2, B1 n^2, A2 m^2, B2 n^2] FP64,
// sigma [E][4] FP64, status [E] int32, tables [E][sys_tab_entries] FP64, the
// same tables in FP32, kinds [E][kMaxN] int8 (the 2 x 2 block markers of TB).
struct SysLayout {
    long nf, ne;
    size_t factors, sigma, status, tab64, tab32, kinds, total;
};
KP_INLINE bool sys_layout(int nc, int n, long E, SysLayout* L) {
    if (nc < 1 || n < 2 || (long)nc * n > kSysMaxM || E < 0) return false;
    const int m = nc * n;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    L->nf = sys_factor_entries(m, n);
    L->ne = sys_tab_entries(m, n);
    size_t o = 0;
    L->factors = o; o += up((size_t)E * L->nf * 8);
    L->sigma = o;   o += up((size_t)E * 4 * 8);
    L->status = o;  o += up((size_t)E * 4);
    L->tab64 = o;   o += up((size_t)E * L->ne * 8);
    L->tab32 = o;   o += up((size_t)E * L->ne * 4);
    L->kinds = o;   o += up((size_t)E * kMaxN);
    L->total = o;
    return true;
}

// Element record of a systems batch: [Jx, Jy, Jx+, Jy+, Jx-, Jy-] (nc x nc
// row-major each; J+ = (J)^+ the outflow part through the high face,
// J- = (-J)^+ through the low face), then nu, alpha, phi, tau, face.
KP_INLINE long sys_rec_len(int nc) { return 6L * nc * nc + 5; }

// Entry (I, J) of the explicit block of one element (rows test, columns trial
// functions; nodal order (component, x, y)): the scalar weak form of
// Sec. 3.4 (eq. adv-kron) with the advection velocity replaced by the flux
// Jacobians, collocated Gauss-Legendre quadrature on [0,1]^2:
//   I (x) diag(w (x) w * c) + tau [-Jx (x) S (x) W - Jy (x) W (x) S
//   + nu I (x) (K (x) W + W (x) K)] + tau [Jx+ (x) l1 l1^T (x) W
//   + Jx- (x) l0 l0^T (x) W + Jy+ (x) W (x) l1 l1^T + Jy- (x) W (x) l0 l0^T]
// (faces only if face != 0), c = 1 + alpha sin(pi x y + phi) at the nodes.
KP_INLINE double sys_block_entry(int nc, int n, long I, long J, const double* rec, const Tables1D& T) {
    const int nn = n * n, q = nc * nc;
    const int ci = (int)(I / nn), i = (int)((I / n) % n), j = (int)(I % n);
    const int cj = (int)(J / nn), k = (int)((J / n) % n), l = (int)(J % n);
    const double nu = rec[6 * q], alpha = rec[6 * q + 1], phi = rec[6 * q + 2], tau = rec[6 * q + 3];
    const bool face = rec[6 * q + 4] != 0.0;
    const int cc = ci * nc + cj;
    const double Jx = rec[cc], Jy = rec[q + cc];
    double v = 0.0;
    if (ci == cj && i == k && j == l) {
        const double c = 1.0 + alpha * sin(3.14159265358979323846 * T.x[i] * T.x[j] + phi);
        v += T.w[i] * T.w[j] * c;
    }
    double t = 0.0;
    if (j == l) t -= Jx * T.S[i * n + k] * T.w[j];
    if (i == k) t -= Jy * T.w[i] * T.S[j * n + l];
    if (ci == cj) {
        if (j == l) t += nu * T.K[i * n + k] * T.w[j];
        if (i == k) t += nu * T.w[i] * T.K[j * n + l];
    }
    if (face) {
        const double Jxp = rec[2 * q + cc], Jyp = rec[3 * q + cc], Jxm = rec[4 * q + cc], Jym = rec[5 * q + cc];
        if (j == l) t += (Jxp * T.l1[i] * T.l1[k] + Jxm * T.l0[i] * T.l0[k]) * T.w[j];
        if (i == k) t += T.w[i] * (Jyp * T.l1[j] * T.l1[l] + Jym * T.l0[j] * T.l0[l]);
    }
    return v + tau * t;
}

KP_INLINE int sys_kmax(int n) {
    const int k = 64;
    return k < n * n ? k : n * n;
}

// work of the tables (tables_sys): six m x m matrices, kMaxN doubles and the
// rotated factors (2 m^2 + 2 n^2)
KP_INLINE long sys_tables_work_doubles(int m, int n) { return 8L * m * m + 2L * n * n + kMaxN; }

// per-element work: Lanczos (n^2 space), the Gram R^T R, the Ritz vectors,
// and the tables' work
KP_INLINE long sys_work_doubles(int m, int n) {
    const long nn = (long)n * n, k = sys_kmax(n);
    return (k + 1) * nn + nn + (k + 2) + 2 * (k + 1) + 2 * k + k * k + 3 * k + 3 + 8 + 2 * k + 4 + nn * nn +
           3 * nn + sys_tables_work_doubles(m, n) + 8;
}
KP_INLINE SetupWork carve_sys(double* p, int m, int n, double** tabwork) {
    const long nn = (long)n * n, k = sys_kmax(n);
    (void)m;
    SetupWork W = {};
    W.L.Q = p; p += (k + 1) * nn;
    W.L.w = p; p += nn;
    W.L.qv = nullptr;
    W.L.h = p; p += k + 2;
    W.L.alpha = p; p += k + 1;
    W.L.beta = p; p += k + 1;
    W.L.d = p; p += k;
    W.L.e = p; p += k;
    W.L.Z = p; p += k * k;
    W.L.sel = p; p += 3 * k;
    W.L.theta = p; p += 3;
    W.L.ctrl = (int*)p; p += 8;
    W.L.rot = p; p += 2 * k;
    W.L.qc = (int*)p; p += 4;
    W.G = p; p += nn * nn;
    W.U = p; p += 3 * nn;
    *tabwork = p;
    return W;
}

// G = R(A)^T R(A) of an explicit (m n) x (m n) block:
// G[(K,K'),(L,L')] = sum_{a,a'} A[a n + K, a' n + K'] A[a n + L, a' n + L']
template <class Team>
KP_HD void sys_right_gram_generic(const Team& tm, int m, int n, const double* A, double* G) {
    const int q2 = n * n;
    const long N = (long)m * n;
    for (int idx = tm.tid(); idx < q2 * q2; idx += tm.size()) {
        const int p = idx / q2, q = idx % q2;
        if (q < p) continue;
        const int K = p / n, K2 = p % n, L = q / n, L2 = q % n;
        double acc = 0.0;
        for (int a = 0; a < m; ++a) {
            const double* ra = A + ((long)a * n + K) * N + K2;
            const double* rb = A + ((long)a * n + L) * N + L2;
            for (int a2 = 0; a2 < m; ++a2) acc += ra[(long)a2 * n] * rb[(long)a2 * n];
        }
        G[(long)p * q2 + q] = acc;
        G[(long)q * q2 + p] = acc;
    }
    tm.sync();
}

template <class Team>
KP_HD void sys_right_gram(const Team& tm, int m, int n, const double* A, double* G) {
    sys_right_gram_generic(tm, m, n, A, G);
}
#if defined(__HIPCC__)
// workgroup form for n^2 <= 64 and 256 threads: rows of R(A) staged in LDS
// 32 at a time (for a fixed a, the rows (a, a0..a0+31) are n runs of 32 n
// consecutive block entries: coalesced loads), every thread accumulating a
// 4 x 4 tile of G in registers
__device__ inline void sys_right_gram(const BlockTeam& tm, int m, int n, const double* A, double* G) {
    const int q2 = n * n;
    if (q2 > 64 || blockDim.x != 256) {
        sys_right_gram_generic(tm, m, n, A, G);
        return;
    }
    __shared__ double Rc[32 * 64];
    const int t = (int)threadIdx.x, ti = t >> 4, tj = t & 15;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    const long N = (long)m * n;
    for (int a = 0; a < m; ++a)
        for (int a0 = 0; a0 < m; a0 += 32) {
            const int kc = m - a0 < 32 ? m - a0 : 32;
            const int span = kc * n;
            const double* base = A + (long)a * n * N + (long)a0 * n;
            for (int idx = t; idx < n * span; idx += 256) {
                const int K = idx / span, rem = idx % span;
                Rc[(rem / n) * q2 + K * n + rem % n] = base[(long)K * N + rem];
            }
            __syncthreads();
            for (int kk = 0; kk < kc; ++kk) {
                const double* row = Rc + kk * q2;
                double ri[4], cj[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    ri[i] = 4 * ti + i < q2 ? row[4 * ti + i] : 0.0;
                    cj[i] = 4 * tj + i < q2 ? row[4 * tj + i] : 0.0;
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] += ri[i] * cj[j];
            }
            __syncthreads();
        }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = 4 * ti + i, c = 4 * tj + j;
            if (r < q2 && c < q2) G[r * q2 + c] = acc[i][j];
        }
    __syncthreads();
}
#endif

// B = sc R(A) x for a right vector x (n x n), B a left vector (m x m)
struct SysLeftOp {
    const OpStream* op;
    template <class Team>
    KP_HD void operator()(const Team& tm, const double* x, double sc, double* B) const {
        op->forward(tm, x, B);
        if (sc != 1.0) {
            for (int t = tm.tid(); t < op->n * op->n; t += tm.size()) B[t] *= sc;
            tm.sync();
        }
    }
    // the map back: y = R(A)^T x for a left vector x (m x m)
    template <class Team>
    KP_HD void forward(const Team& tm, const double* x, double* y) const {
        op->right_factor(tm, x, 1.0, y);
    }
};

// factors and singular values of one element (rank 2): the top right
// singular vectors v_j by Lanczos on the Gram, u_j = R v_j / sigma_j; the sign
// of each pair then puts the largest-magnitude entry of A_j positive.
template <class Team>
KP_HD int setup_sys_element(const Team& tm, int m, int n, const double* block, double* F, double* sigma,
                            SetupWork& W) {
    for (int j = tm.tid(); j < 4; j += tm.size()) sigma[j] = 0.0;
    tm.sync();
    const long ma = (long)m * m, nb = (long)n * n;
    sys_right_gram(tm, m, n, block, W.G);
    OpGram og{n * n, W.G};
    OpStream st{m, n, block, nullptr};
    SysLeftOp lo{&st};
    const long stride = ma + nb;  // A1 -> A2, B1 -> B2
    const int status = ksvd_stage<false>(tm, og, lo, n, 2, sys_kmax(n), nullptr, W, F + ma, stride, F, stride,
                                         m, sigma);
    for (int j = 0; j < 2; ++j) {
        double* A = F + j * stride;
        double* B = A + ma;
        const double sg = canonical_sign(tm, A, m * m, W.L.ctrl + 2);
        if (sg < 0.0) {
            for (long t = tm.tid(); t < nb; t += tm.size()) B[t] = -B[t];
            tm.sync();
        }
    }
    return status;
}

// Column c of (M + shift I)^{-1} for M quasi-upper-triangular (m x m
// row-major; a 2 x 2 diagonal block at rows i - 1, i where M[i][i - 1] != 0),
// by back substitution on e_c; written to out[i m + c].  Returns false on a
// zero pivot or a singular 2 x 2 block.
KP_INLINE bool qt_inverse_col(int m, const double* M, double shift, int c, double* out) {
    int i = m - 1;
    bool ok = true;
    while (i >= 0) {
        if (i >= 1 && M[i * m + i - 1] != 0.0) {
            double r1 = (i - 1 == c) ? 1.0 : 0.0, r2 = (i == c) ? 1.0 : 0.0;
            for (int k = i + 1; k < m; ++k) {
                const double xk = out[k * m + c];
                r1 -= M[(i - 1) * m + k] * xk;
                r2 -= M[i * m + k] * xk;
            }
            const double a = M[(i - 1) * m + i - 1] + shift, b = M[(i - 1) * m + i];
            const double cc = M[i * m + i - 1], d = M[i * m + i] + shift;
            const double det = a * d - b * cc;
            if (det == 0.0) {
                ok = false;
                out[(i - 1) * m + c] = 0.0;
                out[i * m + c] = 0.0;
            } else {
                out[(i - 1) * m + c] = (d * r1 - b * r2) / det;
                out[i * m + c] = (a * r2 - cc * r1) / det;
            }
            i -= 2;
        } else {
            double r = (i == c) ? 1.0 : 0.0;
            for (int k = i + 1; k < m; ++k) r -= M[i * m + k] * out[k * m + c];
            const double piv = M[i * m + i] + shift;
            if (piv == 0.0) {
                ok = false;
                out[i * m + c] = 0.0;
            } else {
                out[i * m + c] = r / piv;
            }
            i -= 1;
        }
    }
    return ok;
}

// Column c of (M + (sr + i si) I)^{-1} for M quasi-upper-triangular as
// above, in complex arithmetic: real parts to outr[i m + c], imaginary parts
// to outi[i m + c].  Returns false on a zero pivot or a singular 2 x 2 block.
KP_INLINE bool qt_inverse_col_c(int m, const double* M, double sr, double si, int c, double* outr, double* outi) {
    // (a + ib) / (x + iy)
    auto cdiv = [](double a, double b, double x, double y, double* re, double* im) {
        const double d = x * x + y * y;
        *re = (a * x + b * y) / d;
        *im = (b * x - a * y) / d;
    };
    int i = m - 1;
    bool ok = true;
    while (i >= 0) {
        if (i >= 1 && M[i * m + i - 1] != 0.0) {
            double r1 = (i - 1 == c) ? 1.0 : 0.0, r1i = 0.0, r2 = (i == c) ? 1.0 : 0.0, r2i = 0.0;
            for (int k = i + 1; k < m; ++k) {
                const double xr = outr[k * m + c], xi = outi[k * m + c];
                const double m1 = M[(i - 1) * m + k], m2 = M[i * m + k];
                r1 -= m1 * xr;
                r1i -= m1 * xi;
                r2 -= m2 * xr;
                r2i -= m2 * xi;
            }
            const double ar = M[(i - 1) * m + i - 1] + sr, b = M[(i - 1) * m + i];
            const double cc = M[i * m + i - 1], dr = M[i * m + i] + sr;
            // det = (a + i si)(d + i si) - b cc
            const double detr = ar * dr - si * si - b * cc, deti = si * (ar + dr);
            if (detr == 0.0 && deti == 0.0) {
                ok = false;
                outr[(i - 1) * m + c] = outi[(i - 1) * m + c] = 0.0;
                outr[i * m + c] = outi[i * m + c] = 0.0;
            } else {
                // x1 = ((d + i si) r1 - b r2) / det, x2 = ((a + i si) r2 - cc r1) / det
                const double n1r = dr * r1 - si * r1i - b * r2, n1i = dr * r1i + si * r1 - b * r2i;
                const double n2r = ar * r2 - si * r2i - cc * r1, n2i = ar * r2i + si * r2 - cc * r1i;
                cdiv(n1r, n1i, detr, deti, &outr[(i - 1) * m + c], &outi[(i - 1) * m + c]);
                cdiv(n2r, n2i, detr, deti, &outr[i * m + c], &outi[i * m + c]);
            }
            i -= 2;
        } else {
            double r = (i == c) ? 1.0 : 0.0, ri = 0.0;
            for (int k = i + 1; k < m; ++k) {
                r -= M[i * m + k] * outr[k * m + c];
                ri -= M[i * m + k] * outi[k * m + c];
            }
            const double pr = M[i * m + i] + sr;
            if (pr == 0.0 && si == 0.0) {
                ok = false;
                outr[i * m + c] = outi[i * m + c] = 0.0;
            } else {
                cdiv(r, ri, pr, si, &outr[i * m + c], &outi[i * m + c]);
            }
            i -= 1;
        }
    }
    return ok;
}

// The angle index k (angle pi k / 8, k < 8) minimising
// kappa_1(-s A1 + c A2) kappa_1(c B1 + s B2) (lowest k on ties); W0, W1, W2:
// m x m scratch, mult: kMaxN doubles.
template <class Team>
KP_HD int sys_rotation_angle(const Team& tm, int m, int n, const double* A1, const double* A2, const double* B1,
                             const double* B2, double* W0, double* W1, double* W2, double* mult, double* sh) {
    const long ma = (long)m * m, nb = (long)n * n;
    const double pi = 3.14159265358979323846;
    double best = -1.0;
    int bestk = 0;
    for (int k = 0; k < 8; ++k) {
        const double c = cos(pi * k / 8.0), sn = sin(pi * k / 8.0);
        for (long t = tm.tid(); t < ma; t += tm.size()) W0[t] = -sn * A1[t] + c * A2[t];
        for (long t = tm.tid(); t < nb; t += tm.size()) W2[t] = c * B1[t] + sn * B2[t];
        tm.sync();
        double score = 1.0;
        for (int q = 0; q < 2; ++q) {
            const int sz = q == 0 ? m : n;
            double* M = q == 0 ? W0 : W2;
            const double nm = norm1(tm, sz, M, sh);
            const bool ok = invert(tm, sz, M, W1, nullptr, mult);
            const double ni = norm1(tm, sz, W1, sh);
            score *= ok ? nm * ni : 1e300;
        }
        if (!(score == score)) score = 1e300;
        if (best < 0.0 || score < best) {
            best = score;
            bestk = k;
        }
    }
    return bestk;
}
#if defined(__HIPCC__)
// kappa_1 = ||M||_1 ||M^-1||_1 of the sz x sz matrix (sz <= 32) whose row i
// lane i of the calling 32-lane group holds in a[]: Gauss-Jordan in place
// with partial pivoting in registers (one row per lane, the pivot row
// broadcast through the group's LDS slot of 32 doubles).  The rows are never
// swapped, so a[] ends as M^-1 with its rows and columns permuted, which
// leaves the largest column sum unchanged.  The same value on every lane of
// the group, 1e300 if a pivot column is zero.
// largest column sum of |row| over the 32-lane group (lane i holding row i,
// inactive lanes zero) for columns < sz: a halving exchange leaves lane l
// with the sum of column l (each step sends the half the partner keeps),
// then a maximum over the lanes.
__device__ __forceinline__ double grp32_max_colsum(const double (&a)[32], bool act, int sz) {
    const int lane = (int)(threadIdx.x & 31);
    double v[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) v[j] = act ? fabs(a[j]) : 0.0;
#pragma unroll
    for (int h = 16; h > 0; h >>= 1) {
        const bool up = (lane & h) != 0;
#pragma unroll
        for (int t = 0; t < h; ++t) {
            const double send = up ? v[t] : v[h + t];
            const double keep = up ? v[h + t] : v[t];
            v[t] = keep + __shfl_xor(send, h, 32);
        }
    }
    double mx = lane < sz ? v[0] : 0.0;
    for (int off = 16; off > 0; off >>= 1) {
        const double o = __shfl_xor(mx, off, 32);
        mx = o > mx ? o : mx;
    }
    return mx;
}

__device__ __forceinline__ double grp32_kappa1(int sz, double (&a)[32], double* sl) {
    const int i = (int)(threadIdx.x & 31);
    const bool act = i < sz;
    const double nm = grp32_max_colsum(a, act, sz);
    bool used = false, ok = true;
#pragma unroll 1
    for (int k = 0; k < sz; ++k) {
        double ak = 0.0;
#pragma unroll
        for (int j = 0; j < 32; ++j)
            if (j == k) ak = a[j];
        double v = (act && !used) ? fabs(ak) : -1.0;
        int p = i;
        for (int off = 16; off > 0; off >>= 1) {
            const double ov = __shfl_xor(v, off, 32);
            const int op = __shfl_xor(p, off, 32);
            if (ov > v || (ov == v && op < p)) {
                v = ov;
                p = op;
            }
        }
        const bool sing = !(v > 0.0);
        if (sing) ok = false;
        const bool piv = act && !sing && i == p;
        if (piv) {
            // the pivot row: column k becomes 1 / pivot, the rest scaled by it
            const double inv = 1.0 / ak;
#pragma unroll
            for (int j = 0; j < 32; ++j) {
                a[j] = (j == k) ? inv : a[j] * inv;
                sl[j] = a[j];
            }
            used = true;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (act && !sing && !piv) {
            // every other row: subtract its multiple; column k becomes -f / pivot
#pragma unroll
            for (int j = 0; j < 32; ++j) a[j] = (j == k) ? -ak * sl[j] : a[j] - ak * sl[j];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    const double ni = grp32_max_colsum(a, act, sz);
    const double kap = nm * ni;
    return (ok && kap == kap) ? kap : 1e300;
}

// The angle search of tables_sys for one element's factors F (as stored:
// A1, B1, A2, B2) by a workgroup of 256 threads: the eight angles at once, one
// 32-lane group each, the balanced rotated factors built in registers and
// each candidate inverted there.  Returns the angle index on every thread.
__device__ inline int sys_angle_search_grp(const BlockTeam& tm, int m, int n, const double* F) {
    __shared__ double slots[8 * 32];
    __shared__ double score[8];
    const long ma = (long)m * m, nb = (long)n * n;
    const double *F1 = F, *G1 = F + ma, *F2 = F + ma + nb, *G2 = F + 2 * ma + nb;
    double p1 = 0.0, p2 = 0.0;
    for (long t = threadIdx.x; t < ma; t += blockDim.x) {
        p1 += F1[t] * F1[t];
        p2 += F2[t] * F2[t];
    }
    const double s1 = sqrt(tm.sum(p1)), s2 = sqrt(tm.sum(p2));
    const double a1 = s1 > 0.0 ? s1 : 1.0, a2 = s2 > 0.0 ? s2 : 1.0;
    const int g = (int)(threadIdx.x >> 5), i = (int)(threadIdx.x & 31);
    const double pi = 3.14159265358979323846;
    const double c = cos(pi * g / 8.0), sn = sin(pi * g / 8.0);
    double a[32];
#pragma unroll
    for (int j = 0; j < 32; ++j)
        a[j] = (i < m && j < m) ? -sn * (F1[i * m + j] / a1) + c * (F2[i * m + j] / a2) : 0.0;
    const double kl = grp32_kappa1(m, a, slots + g * 32);
#pragma unroll
    for (int j = 0; j < 32; ++j)
        a[j] = (i < n && j < n) ? c * (G1[i * n + j] * a1) + sn * (G2[i * n + j] * a2) : 0.0;
    const double kr = grp32_kappa1(n, a, slots + g * 32);
    double sc = kl * kr;
    if (!(sc == sc) || kl >= 1e300 || kr >= 1e300) sc = 1e300;
    if (i == 0) score[g] = sc;
    tm.sync();
    int bestk = 0;
    for (int k = 1; k < 8; ++k)
        if (score[k] < score[bestk]) bestk = k;
    tm.sync();
    return bestk;
}
#endif

// inversion data of one element.  work: sys_tables_work_doubles(m, n)
// doubles; sh: kMaxN + 8 shared doubles; rot_k: the pair rotation's angle
// index if already chosen (sys_angle_search_grp), else -1 (searched here).
// Returns the element status bits (2 singular factor, 4 Schur not
// converged, 8 non-finite tables).
// Real Schur form of an s x s matrix (s <= 32) for the tables.  Its
// reflector loops span at most s lanes, so on a workgroup team the first wave
// runs the QR alone, with wave barriers in place of the workgroup barriers of
// its thousands of dependent steps, and the other waves wait at one barrier.
// flag: one shared double.
template <class Team>
KP_HD bool sys_schur(const Team& tm, int s, double* H, double* Q, double* sh, double* flag) {
    (void)flag;
    return real_schur(tm, s, H, Q, sh);
}
#if defined(__HIPCC__)
__device__ inline bool sys_schur(const BlockTeam& tm, int s, double* H, double* Q, double* sh, double* flag) {
    if (tm.group() == 0) {
        WaveTeam wt;
        const bool ok = real_schur(wt, s, H, Q, sh);
        if (wt.leader()) *flag = ok ? 1.0 : 0.0;
    }
    tm.sync();
    const bool ok = *flag != 0.0;
    tm.sync();
    return ok;
}
#endif

template <class Team>
KP_HD int tables_sys(const Team& tm, int m, int n, const double* F, double* tab, int8_t* kinds, double* work,
                     double* sh, int rot_k = -1) {
    const long ma = (long)m * m, nb = (long)n * n;
    const SysTab o = sys_tab(m, n);
    double* W0 = work;
    double* W1 = W0 + ma;
    double* W2 = W1 + ma;
    double* W3 = W2 + ma;
    double* W4 = W3 + ma;
    double* W5 = W4 + ma;
    double* mult = W5 + ma;
    int status = 0;
    // Pair rotation before inversion: A1 (x) B1 + A2 (x) B2 is unchanged when
    // (A1, A2) and (B1, B2) are rotated by the same angle after balancing the
    // norms within each term.  The route inverts A2 and B1, which can be
    // nearly singular while P is well conditioned, so the angle (one of 8 in
    // [0, pi)) that minimises kappa_1(A2') kappa_1(B1') is used.  The stored
    // factors stay the KSVD's.
    double* A1 = mult + kMaxN;
    double* A2 = A1 + ma;
    double* B1 = A2 + ma;
    double* B2 = B1 + nb;
    {
        const double *F1 = F, *G1 = F + ma, *F2 = F + ma + nb, *G2 = F + 2 * ma + nb;
        double p1 = 0.0, p2 = 0.0;
        for (long t = tm.tid(); t < ma; t += tm.size()) {
            p1 += F1[t] * F1[t];
            p2 += F2[t] * F2[t];
        }
        const double s1 = sqrt(tm.sum(p1)), s2 = sqrt(tm.sum(p2));
        const double a1 = s1 > 0.0 ? s1 : 1.0, a2 = s2 > 0.0 ? s2 : 1.0;
        for (long t = tm.tid(); t < ma; t += tm.size()) {
            A1[t] = F1[t] / a1;
            A2[t] = F2[t] / a2;
        }
        for (long t = tm.tid(); t < nb; t += tm.size()) {
            B1[t] = G1[t] * a1;
            B2[t] = G2[t] * a2;
        }
        tm.sync();
        const double pi = 3.14159265358979323846;
        const int bestk = rot_k >= 0 ? rot_k : sys_rotation_angle(tm, m, n, A1, A2, B1, B2, W0, W1, W2, mult, sh);
        const double c = cos(pi * bestk / 8.0), sn = sin(pi * bestk / 8.0);
        for (long t = tm.tid(); t < ma; t += tm.size()) {
            const double l1 = A1[t], l2 = A2[t];
            A1[t] = c * l1 + sn * l2;
            A2[t] = -sn * l1 + c * l2;
        }
        for (long t = tm.tid(); t < nb; t += tm.size()) {
            const double r1 = B1[t], r2 = B2[t];
            B1[t] = c * r1 + sn * r2;
            B2[t] = -sn * r1 + c * r2;
        }
        tm.sync();
    }
    // (size, inverted factor, other factor, L, Q, T) for the two sides
    for (int side = 0; side < 2; ++side) {
        const int s = side == 0 ? m : n;
        const long ss = (long)s * s;
        const double* Finv = side == 0 ? A2 : B1;
        const double* Foth = side == 0 ? A1 : B2;
        for (long t = tm.tid(); t < ss; t += tm.size()) W0[t] = Finv[t];
        tm.sync();
        if (!invert(tm, s, W0, W1, nullptr, mult)) status |= 2;
        mm(tm, s, W1, Foth, W2);                              // C = Finv^-1 Foth
        if (!sys_schur(tm, s, W2, W3, sh, mult)) status |= 4;  // W2 <- T, W3 <- Q
        mtm(tm, s, W3, W1, W4);                               // L = Q^T Finv^-1
        double* L = tab + (side == 0 ? o.LA : o.LB);
        double* Q = tab + (side == 0 ? o.QA : o.QB);
        double* T = tab + (side == 0 ? o.TA : o.TB);
        for (long t = tm.tid(); t < ss; t += tm.size()) {
            L[t] = W4[t];
            Q[t] = W3[t];
            T[t] = W2[t];
        }
        tm.sync();
    }
    const double* TA = tab + o.TA;
    const double* TB = tab + o.TB;
    for (int j = tm.tid(); j < n; j += tm.size()) {
        int kd = 0;
        if (j > 0 && TB[j * n + j - 1] != 0.0) kd = 2;
        if (j + 1 < n && TB[(j + 1) * n + j] != 0.0) kd = 1;
        kinds[j] = (int8_t)kd;
    }
    tm.sync();
    // column inverses of the sweep.  Every matrix inverted here is TA plus a
    // (real or complex) multiple of I, quasi-upper-triangular with the 2 x 2
    // diagonal blocks of TA, so each column of the inverse is one back
    // substitution, independent of the others.
    double* N = tab + o.N;
    double* TAw = W5;
    for (long t = tm.tid(); t < ma; t += tm.size()) TAw[t] = TA[t];
    tm.sync();
    double sing = 0.0;
    for (int t = tm.tid(); t < n * m; t += tm.size()) {
        const int j = t / m, c = t % m;
        if (kinds[j] != 0) continue;
        if (!qt_inverse_col(m, TAw, TB[j * n + j], c, N + (long)j * ma)) sing = 1.0;
    }
    tm.sync();
    // a 2 x 2 block of TB at (j - 1, j), [[p, q], [sv, p]] with q sv < 0: its
    // two columns solve (TA + pI) y1 + q y2 = f1, sv y1 + (TA + pI) y2 = f2,
    // i.e. (TA + (p - i w) I) (y1 + i y2 / g) = f1 + i f2 / g with
    // w = sqrt(-q sv), g = w / q.  The complex inverse K = Kr + i Ki goes to
    // the N slots j - 1 (Kr) and j (Ki); its conditioning is that of the
    // shifted TA itself.
    for (int t = tm.tid(); t < n * m; t += tm.size()) {
        const int j = t / m, c = t % m;
        if (kinds[j] != 2) continue;
        const double p = TB[j * n + j], qs = TB[(j - 1) * n + j] * TB[j * n + j - 1];
        if (!(qs < 0.0)) {
            sing = 1.0;
            continue;
        }
        if (!qt_inverse_col_c(m, TAw, p, -sqrt(-qs), c, N + (long)(j - 1) * ma, N + (long)j * ma)) sing = 1.0;
    }
    tm.sync();
    if (tm.max(sing) != 0.0) status |= 2;
    double bad = 0.0;
    for (long t = tm.tid(); t < sys_tab_entries(m, n); t += tm.size())
        if (!(fabs(tab[t]) < 1e300)) bad = 1.0;
    if (tm.max(bad) != 0.0) status |= 8;
    return status;
}

// out[i os] = sum_a M[i m + a] x[a xs] for i < m (M m x m row-major)
template <class Team, typename T, typename TT>
KP_HD void sys_matvec(const Team& tm, int m, const TT* M, const T* x, int xs, T* out, int os) {
    for (int i = tm.tid(); i < m; i += tm.size()) {
        T acc = (T)0;
        for (int a = 0; a < m; ++a) acc += (T)M[i * m + a] * x[a * xs];
        out[i * os] = acc;
    }
    tm.sync();
}
#if defined(__HIPCC__)
// workgroup form: g consecutive lanes per row (g a power of two, g m <= the
// workgroup size), lane p of a row reading M[i m + p + g q], so that the g
// lanes of a row read g consecutive entries per step; the partial sums are
// combined across the g lanes by shuffles
template <typename T, typename TT>
__device__ void sys_matvec(const BlockTeam& tm, int m, const TT* M, const T* x, int xs, T* out, int os) {
    int g = 64;
    while (g > 1 && g * m > (int)blockDim.x) g >>= 1;
    const int t = (int)threadIdx.x, i = t / g, p = t % g;
    T acc = (T)0;
    if (i < m)
        for (int a = p; a < m; a += g) acc += (T)M[i * m + a] * x[a * xs];
    for (int o = g >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (i < m && p == 0) out[i * os] = acc;
    tm.sync();
}
#endif

// X (m x n, row-major) <- P^{-1} X.  Y: m n scratch, Hs: 2 m scratch.
template <class Team, typename T, typename TT>
KP_HD void apply_sys(const Team& tm, int m, int n, const TT* tab, const int8_t* kinds, T* X, T* Y, T* Hs) {
    const SysTab o = sys_tab(m, n);
    const TT* LA = tab + o.LA;
    const TT* LB = tab + o.LB;
    const TT* QA = tab + o.QA;
    const TT* QB = tab + o.QB;
    const TT* TA = tab + o.TA;
    const TT* TB = tab + o.TB;
    const TT* N = tab + o.N;
    const long mm = (long)m * m;
    // Y = LA X; X = Y LB^T  (F in X)
    for (int t = tm.tid(); t < m * n; t += tm.size()) {
        const int i = t / n, k = t % n;
        T acc = (T)0;
        for (int a = 0; a < m; ++a) acc += (T)LA[i * m + a] * X[a * n + k];
        Y[t] = acc;
    }
    tm.sync();
    for (int t = tm.tid(); t < m * n; t += tm.size()) {
        const int i = t / n, k = t % n;
        T acc = (T)0;
        for (int b = 0; b < n; ++b) acc += Y[i * n + b] * (T)LB[k * n + b];
        X[t] = acc;
    }
    tm.sync();
    // TA S + S TB^T = F: columns j from n - 1 down (S in Y)
    T* F = X;
    T* S = Y;
    int j = n - 1;
    while (j >= 0) {
        const int kd = kinds[j];
        if (kd != 2) {
            sys_matvec(tm, m, N + (long)j * mm, F + j, n, S + j, n);
            for (int t = tm.tid(); t < m * j; t += tm.size()) {
                const int k = t % j, i = t / j;
                F[i * n + k] -= (T)TB[k * n + j] * S[i * n + j];
            }
            tm.sync();
            --j;
        } else {
            // y1 = Kr f1 - Ki f2 / g, y2 = g Ki f1 + Kr f2 (K the complex inverse
            // of the block, g = w / q)
            const int j1 = j - 1;
            const T q = (T)TB[j1 * n + j], sv = (T)TB[j * n + j1];
            const T g = sqrt(-q * sv) / q;
            const TT* Kr = N + (long)j1 * mm;
            const TT* Ki = N + (long)j * mm;
            sys_matvec(tm, m, Kr, F + j1, n, S + j1, n);
            sys_matvec(tm, m, Kr, F + j, n, S + j, n);
            sys_matvec(tm, m, Ki, F + j, n, Hs, 1);
            sys_matvec(tm, m, Ki, F + j1, n, Hs + m, 1);
            for (int i = tm.tid(); i < m; i += tm.size()) {
                S[i * n + j1] -= Hs[i] / g;
                S[i * n + j] += g * Hs[m + i];
            }
            tm.sync();
            for (int t = tm.tid(); t < m * j1; t += tm.size()) {
                const int k = t % j1, i = t / j1;
                F[i * n + k] -= (T)TB[k * n + j1] * S[i * n + j1] + (T)TB[k * n + j] * S[i * n + j];
            }
            tm.sync();
            j -= 2;
        }
    }
    // X = QA S; Y = X QB^T; result back in X
    for (int t = tm.tid(); t < m * n; t += tm.size()) {
        const int i = t / n, k = t % n;
        T acc = (T)0;
        for (int a = 0; a < m; ++a) acc += (T)QA[i * m + a] * S[a * n + k];
        F[t] = acc;
    }
    tm.sync();
    for (int t = tm.tid(); t < m * n; t += tm.size()) {
        const int i = t / n, k = t % n;
        T acc = (T)0;
        for (int b = 0; b < n; ++b) acc += F[i * n + b] * (T)QB[k * n + b];
        S[t] = acc;
    }
    tm.sync();
    for (int t = tm.tid(); t < m * n; t += tm.size()) X[t] = S[t];
    tm.sync();
}

}  // namespace kp
