// Rank-3 2D apply: z = P3^{-1} r with P3 = A1 (x) B1 + A2 (x) B2 + A3 (x) B3.
//
// The paper's direct inverse covers two Kronecker terms only (Sec. 4.2: more
// terms have no Schur-form shortcut).  P3 is solved per element by flexible
// GMRES(m), preconditioned by the rank-2 Schur-route apply built from the
// first two terms (the best rank-2 approximation, so the preconditioned
// operator is a small perturbation of the identity).  The Kronecker products
// and the Arnoldi process run in FP64; the rank-2 apply runs in the requested
// precision.  Because the flexible variant keeps every preconditioned vector,
// the residual the iteration reports is that of the returned iterate, so a
// lower-precision inner apply costs iterations, not accuracy.
#pragma once

#include "elem_ops.h"

namespace kp {

// w = P3 u for one element.  F: the six factors A1,B1,A2,B2,A3,B3 (n x n,
// row-major); u, w: n^2 (row-major X[i][k] = x[i*n + k], so (A (x) B) x is
// A X B^T); tmp: 3 n^2.  The inner loops are unrolled by eight so that a
// lane's factor loads are in flight together (the summation order is kept).
template <class Team>
KP_HD void kron3_apply(const Team& tm, int n, const double* F, const double* u, double* w,
                       double* tmp) {
    const int nn = n * n;
    // tmp_j[k][l] = sum_q U[k][q] B_j[l][q]
    for (int t = tm.tid(); t < 3 * nn; t += tm.size()) {
        const int j = t / nn, k = (t % nn) / n, l = t % n;
        const double* B = F + (2 * j + 1) * nn;
        double s = 0.0;
#pragma unroll 8
        for (int q = 0; q < n; ++q) s += u[k * n + q] * B[l * n + q];
        tmp[t] = s;
    }
    tm.sync();
    // w[i][l] = sum_j sum_k A_j[i][k] tmp_j[k][l]
    for (int t = tm.tid(); t < nn; t += tm.size()) {
        const int i = t / n, l = t % n;
        double s = 0.0;
        for (int j = 0; j < 3; ++j) {
            const double* A = F + 2 * j * nn;
#pragma unroll 8
            for (int k = 0; k < n; ++k) s += A[i * n + k] * tmp[j * nn + k * n + l];
        }
        w[t] = s;
    }
    tm.sync();
}

KP_INLINE int rank3_work_doubles(int n, int m) { return (2 * m + 6) * n * n; }
KP_INLINE int rank3_small_doubles(int m) { return (m + 1) * m + 4 * (m + 1) + 8; }

// Inner relative residual targets per apply precision (FP64, FP32, BF16, split BF16).
KP_INLINE double rank3_rtol(int prec) {
    return prec == 0 ? 1e-13 : prec == 1 ? 1e-10 : prec == 2 ? 1e-6 : 1e-9;
}
constexpr int kRank3MaxIters = 200;

// z = P3^{-1} r.  tab / kinds: rank-2 apply tables; work: rank3_work_doubles;
// tw: 3 n^2 of T (the rank-2 apply's tensors); small: rank3_small_doubles.
// Returns the number of inner iterations, negated if the target was not met.
template <class Team, typename T, typename TT, class Rnd>
KP_HD int rank3_solve(const Team& tm, int n, const double* F, const TT* tab, const int8_t* kinds,
                      const double* r, double* z, double* work, T* tw, double* small, int m,
                      double rtol, int maxit, Rnd rnd) {
    const int nn = n * n;
    double* V = work;                   // (m + 1) n^2
    double* Z = V + (m + 1) * nn;       // m n^2
    double* x = Z + m * nn;             // n^2
    double* w = x + nn;                 // n^2
    double* tmp = w + nn;               // 3 n^2
    double* H = small;                  // (m + 1) m, column k at H[k * (m + 1)]
    double* g = H + (m + 1) * m;        // m + 1
    double* cs = g + (m + 1);           // m + 1
    double* sn = cs + (m + 1);          // m + 1
    double* h = sn + (m + 1);           // m + 1 (dot products of one pass)
    double* sc = h + (m + 1);           // scalars shared by the team
    T* X = tw;
    T* Y = tw + nn;
    T* Hs = tw + 2 * nn;

    double p = 0.0;
    for (int t = tm.tid(); t < nn; t += tm.size()) {
        x[t] = 0.0;
        p += r[t] * r[t];
    }
    const double beta0 = sqrt(tm.sum(p));  // the sum ends with a barrier
    if (beta0 == 0.0) {
        for (int t = tm.tid(); t < nn; t += tm.size()) z[t] = 0.0;
        tm.sync();
        return 0;
    }
    const double target = rtol * beta0;
    int iters = 0;
    bool converged = false;
    for (;;) {
        // w = r - P3 x (x = 0 on the first cycle)
        if (iters == 0) {
            for (int t = tm.tid(); t < nn; t += tm.size()) w[t] = r[t];
            tm.sync();
        } else {
            kron3_apply(tm, n, F, x, w, tmp);
            for (int t = tm.tid(); t < nn; t += tm.size()) w[t] = r[t] - w[t];
            tm.sync();
        }
        p = 0.0;
        for (int t = tm.tid(); t < nn; t += tm.size()) p += w[t] * w[t];
        const double beta = sqrt(tm.sum(p));
        if (beta <= target) {
            converged = true;
            break;
        }
        if (iters >= maxit) break;
        for (int t = tm.tid(); t < nn; t += tm.size()) V[t] = w[t] / beta;
        for (int t = tm.tid(); t < m + 1; t += tm.size()) g[t] = t == 0 ? beta : 0.0;
        tm.sync();
        int k = 0;
        while (k < m && iters < maxit) {
            // Z_k = M V_k (rank-2 apply in the apply precision)
            for (int t = tm.tid(); t < nn; t += tm.size()) X[t] = (T)V[k * nn + t];
            tm.sync();
            apply_tensor(tm, 2, n, tab, kinds, X, Y, Hs, rnd);
            for (int t = tm.tid(); t < nn; t += tm.size()) Z[k * nn + t] = (double)X[t];
            tm.sync();
            kron3_apply(tm, n, F, Z + k * nn, w, tmp);
            // classical Gram-Schmidt, twice
            double* Hk = H + k * (m + 1);
            for (int t = tm.tid(); t < m + 1; t += tm.size()) Hk[t] = 0.0;
            tm.sync();
            for (int pass = 0; pass < 2; ++pass) {
                tm.dots(V, nn, k + 1, w, nn, h);
                for (int t = tm.tid(); t < nn; t += tm.size()) {
                    double s = w[t];
                    for (int i = 0; i <= k; ++i) s -= h[i] * V[i * nn + t];
                    w[t] = s;
                }
                for (int i = tm.tid(); i <= k; i += tm.size()) Hk[i] += h[i];
                tm.sync();
            }
            p = 0.0;
            for (int t = tm.tid(); t < nn; t += tm.size()) p += w[t] * w[t];
            const double hk1 = sqrt(tm.sum(p));
            const double inv = hk1 > 0.0 ? 1.0 / hk1 : 0.0;
            for (int t = tm.tid(); t < nn; t += tm.size()) V[(k + 1) * nn + t] = w[t] * inv;
            if (tm.leader()) {
                Hk[k + 1] = hk1;
                // previous rotations, then a new one that zeroes H[k+1][k]
                for (int i = 0; i < k; ++i) {
                    const double a = Hk[i], b = Hk[i + 1];
                    Hk[i] = cs[i] * a + sn[i] * b;
                    Hk[i + 1] = -sn[i] * a + cs[i] * b;
                }
                const double a = Hk[k], b = Hk[k + 1];
                const double rr = sqrt(a * a + b * b);
                const double c = rr > 0.0 ? a / rr : 1.0, s = rr > 0.0 ? b / rr : 0.0;
                cs[k] = c;
                sn[k] = s;
                Hk[k] = rr;
                Hk[k + 1] = 0.0;
                g[k + 1] = -s * g[k];
                g[k] = c * g[k];
                sc[0] = fabs(g[k + 1]);
            }
            tm.sync();
            ++k;
            ++iters;
            if (sc[0] <= target || hk1 == 0.0) break;
        }
        // y = H(0:k, 0:k)^{-1} g(0:k) into h, then x += Z y
        if (tm.leader()) {
            for (int i = k - 1; i >= 0; --i) {
                double s = g[i];
                for (int j = i + 1; j < k; ++j) s -= H[j * (m + 1) + i] * h[j];
                const double d = H[i * (m + 1) + i];
                h[i] = d != 0.0 ? s / d : 0.0;
            }
        }
        tm.sync();
        for (int t = tm.tid(); t < nn; t += tm.size()) {
            double s = x[t];
            for (int j = 0; j < k; ++j) s += h[j] * Z[j * nn + t];
            x[t] = s;
        }
        tm.sync();
    }
    for (int t = tm.tid(); t < nn; t += tm.size()) z[t] = x[t];
    tm.sync();
    return converged ? iters : -iters - 1;
}

}  // namespace kp
