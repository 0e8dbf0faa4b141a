// Blocks of nc-component systems (2D): KSVD with nc n x nc n first factors
// (the component index grouped with x; Sec. 5.3), the inversion data and the
// apply of the Kronecker-sum inverse.
//
// Nodal vectors are ordered (component, x, y), component slowest; the block
// is explicit, (m n) x (m n) row-major with m = nc n.  Its rearrangement R(A)
// is m^2 x n^2 (rows: pairs of (component, x) indices; columns: pairs of y
// indices).  Setup: Lanczos (Alg. 2) on the smaller Gram R^T R, then
// A_j = sqrt(sigma_j) u_j (m x m), B_j = sqrt(sigma_j) v_j (n x n).  Inversion data (Alg. 5): C1 =
// A2^-1 A1 (m x m), C2 = B1^-1 B2 (n x n), real Schur forms C1 = QA TA QA^T,
// C2 = QB TB QB^T, LA = QA^T A2^-1, LB = QB^T B1^-1, and the column inverses
// N_j = (TA + t_jj I)^-1 (m x m) of the quasi-triangular Sylvester sweep over
// the n columns of TB (for a 2 x 2 block of TB, ((TA + pI)^2 - qs I)^-1).
// Apply: X (m x n) -> LA X LB^T -> Sylvester TA Y + Y TB^T = F -> QA Y QB^T.
#pragma once

#include "elem_ops.h"

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

KP_INLINE int sys_kmax(int n) {
    const int k = 64;
    return k < n * n ? k : n * n;
}

// per-element work: Lanczos (n^2 space), the Gram R^T R, the Ritz vectors,
// and six m x m matrices and kMaxN doubles for the tables
KP_INLINE long sys_work_doubles(int m, int n) {
    const long nn = (long)n * n, mm = (long)m * m, k = sys_kmax(n);
    return (k + 1) * nn + nn + (k + 2) + 2 * (k + 1) + 2 * k + k * k + 3 * k + 3 + 8 + 2 * k + 4 + nn * nn +
           3 * nn + 6 * mm + kMaxN + 8;
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
KP_HD void sys_right_gram(const Team& tm, int m, int n, const double* A, double* G) {
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

// inversion data of one element.  work: 6 m^2 + kMaxN doubles; sh: kMaxN + 8
// shared doubles.  Returns the element status bits (2 singular factor, 4
// Schur not converged, 8 non-finite tables).
template <class Team>
KP_HD int tables_sys(const Team& tm, int m, int n, const double* F, double* tab, int8_t* kinds, double* work,
                     double* sh) {
    const long ma = (long)m * m, nb = (long)n * n;
    const SysTab o = sys_tab(m, n);
    const double *A1 = F, *B1 = F + ma, *A2 = F + ma + nb, *B2 = F + 2 * ma + nb;
    double* W0 = work;
    double* W1 = W0 + ma;
    double* W2 = W1 + ma;
    double* W3 = W2 + ma;
    double* W4 = W3 + ma;
    double* W5 = W4 + ma;
    double* mult = W5 + ma;
    int status = 0;
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
        if (!real_schur(tm, s, W2, W3, sh)) status |= 4;      // W2 <- T, W3 <- Q
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
    double* N = tab + o.N;
    for (int j = 0; j < n; ++j) {
        const int kd = kinds[j];
        if (kd == 1) continue;  // filled with its partner
        if (kd == 0) {
            const double tj = TB[j * n + j];
            for (long t = tm.tid(); t < ma; t += tm.size()) W0[t] = TA[t] + ((t / m == t % m) ? tj : 0.0);
            tm.sync();
        } else {
            const double p = TB[j * n + j], q = TB[(j - 1) * n + j], sv = TB[j * n + j - 1];
            for (long t = tm.tid(); t < ma; t += tm.size()) W4[t] = TA[t] + ((t / m == t % m) ? p : 0.0);
            tm.sync();
            mm(tm, m, W4, W4, W5);
            for (long t = tm.tid(); t < ma; t += tm.size()) W0[t] = W5[t] - ((t / m == t % m) ? q * sv : 0.0);
            tm.sync();
        }
        if (!invert(tm, m, W0, W1, nullptr, mult)) status |= 2;
        for (long t = tm.tid(); t < ma; t += tm.size()) {
            N[(long)j * ma + t] = W1[t];
            if (kd == 2) N[(long)(j - 1) * ma + t] = W1[t];
        }
        tm.sync();
    }
    double bad = 0.0;
    for (long t = tm.tid(); t < sys_tab_entries(m, n); t += tm.size())
        if (!(fabs(tab[t]) < 1e300)) bad = 1.0;
    if (tm.max(bad) != 0.0) status |= 8;
    return status;
}

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
            const TT* Nj = N + (long)j * mm;
            for (int i = tm.tid(); i < m; i += tm.size()) {
                T acc = (T)0;
                for (int a = 0; a < m; ++a) acc += (T)Nj[i * m + a] * F[a * n + j];
                S[i * n + j] = acc;
            }
            tm.sync();
            for (int t = tm.tid(); t < m * j; t += tm.size()) {
                const int k = t % j, i = t / j;
                F[i * n + k] -= (T)TB[k * n + j] * S[i * n + j];
            }
            tm.sync();
            --j;
        } else {
            const int j1 = j - 1;
            const T p = (T)TB[j * n + j], q = (T)TB[j1 * n + j], sv = (T)TB[j * n + j1];
            const TT* Nj = N + (long)j * mm;
            for (int i = tm.tid(); i < m; i += tm.size()) {
                T a1 = (T)0, a2 = (T)0;
                for (int a = 0; a < m; ++a) {
                    const T ta = (T)TA[i * m + a];
                    a1 += ta * F[a * n + j1];
                    a2 += ta * F[a * n + j];
                }
                const T g1 = F[i * n + j1], g2 = F[i * n + j];
                Hs[i] = a1 + p * g1 - q * g2;
                Hs[m + i] = a2 + p * g2 - sv * g1;
            }
            tm.sync();
            for (int t = tm.tid(); t < 2 * m; t += tm.size()) {
                const int h = t / m, i = t % m;
                T acc = (T)0;
                for (int a = 0; a < m; ++a) acc += (T)Nj[i * m + a] * Hs[h * m + a];
                S[i * n + (h ? j : j1)] = acc;
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
