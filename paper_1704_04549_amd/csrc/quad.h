// General (non-collocated) elements: the rearranged block's Gram operator
// R(A) R(A)^T in closed form from quadrature data (Sec. 3.4.1, eq.
// jac-entries; Sec. 4.2.1 and Sec. 4.3.2, the shuffled products).
//
// A general element carries its coefficients at mu >= n Gauss-Legendre
// points per axis of [0,1]: the mass coefficient c, the flux-Jacobian
// components a_i, a second-order coefficient nu, and the upwind face
// coefficients g_f at each face's own points.  Its block is a sum of terms
//   A_t = (L_x (x) L_y [(x) L_z])^T diag(f_t) (R_x (x) R_y [(x) R_z]),
// one pair (L, R) of point-by-basis matrices per axis, of five types:
//   PP (Phi, Phi), dP (dPhi, Phi), dd (dPhi, dPhi), l0 (phi(0), phi(0)),
//   l1 (phi(1), phi(1))   (the last two have a single point),
// and a coefficient tensor f_t over the product of the axes' points, weights
// and tau included:
//   mass (PP,PP,PP)  w w w c;   advection on axis i (dP on i)  -tau w w w a_i;
//   second order on axis i (dd on i)  tau w w w nu;
//   face x-/x+ (l0/l1 on x)  tau w w g_f (and likewise on y, z).
// Rearranged (rows: pairs (test, trial) of the first axis; columns: those of
// the other axes), each term is X_p^T F Y, with X_p[alpha, (a,c)] =
// L_p[alpha, a] R_p[alpha, c].  Every Gram product X_p X_q^T is a small
// mu_p x mu_q matrix, K_pq = (L_p L_q^T) o (R_p R_q^T) (Hadamard product),
// the same for every element of an (n, mu) pair.  So R R^T x needs only
// products with the coefficient tensors and the K_pq, O(terms mu^3) per
// Lanczos step in 3D, instead of the O(n^4 mu) of two shuffled products
// through a right vector of length n^4.
//
// 3D stage 1 (A ~ A1 (x) D1): x lives on the x-axis pairs (n^2); the terms
// are grouped by their (y, z) types into nine groups g, and
//   q_p = X_p x;  S_g = sum_{t in g} f_t x_alpha q_{tx(t)};
//   W_h = sum_g K_Y[ty(g), ty(h)]^T S_g K_Z[tz(g), tz(h)];
//   Q_p = sum_{t: tx(t) = p} f_t . W_{g(t)} over (beta, gamma);
//   R R^T x = sum_p X_p^T Q_p.
// The right factor R^T u is kept in that factored form: D1 = sum_g (Y_g (x)
// Z_g)-structured with coefficient matrices S_g, itself a general 2D block
// (the groups as its terms) for the rank-2 stage 2.
// 2D (and 3D stage 2): terms (tx, ty, F_t), F_t mu_tx x mu_ty;
//   q_p = X_p x;  S_y = sum_{t: ty(t) = y} F_t^T q_{tx(t)};
//   W_y' = sum_y K[y][y']^T S_y;  Q_p = sum_{t: tx(t) = p} F_t W_{ty(t)};
//   R R^T x = sum_p X_p^T Q_p;  R^T x = sum_y Y_y^T S_y.
#pragma once

#include "elem_ops.h"

namespace kp {

constexpr int kQuadMaxMu = kMaxN;
constexpr int kQuadTypes = 5;  // PP, dP, dd, l0, l1
constexpr int kQuadTerms2 = 9;
constexpr int kQuadTerms3 = 13;
constexpr int kQuadGroups3 = 9;

// 1D tables of an (n, mu) pair (host-computed): the quadrature weights, the
// Lagrange basis on the n Gauss-Legendre nodes and its derivative at the mu
// points, phi(0), phi(1), and the pair Grams K[p][q] (mu_p x mu_q, row-major
// with leading dimension kQuadMaxMu).
struct QuadTables {
    int n, mu;
    double w[kQuadMaxMu];
    double Phi[kQuadMaxMu * kMaxN];   // [alpha * n + j]
    double dPhi[kQuadMaxMu * kMaxN];
    double l0[kMaxN], l1[kMaxN];
    double K[kQuadTypes * kQuadTypes * kQuadMaxMu * kQuadMaxMu];
};

KP_INLINE int qmu(const QuadTables& Q, int type) { return type >= 3 ? 1 : Q.mu; }
KP_INLINE double qL(const QuadTables& Q, int type, int alpha, int a) {
    const int n = Q.n;
    return type == 0 ? Q.Phi[alpha * n + a]
           : type <= 2 ? Q.dPhi[alpha * n + a]
           : type == 3 ? Q.l0[a]
                       : Q.l1[a];
}
KP_INLINE double qR(const QuadTables& Q, int type, int alpha, int c) {
    const int n = Q.n;
    return type <= 1 ? Q.Phi[alpha * n + c] : type == 2 ? Q.dPhi[alpha * n + c] : type == 3 ? Q.l0[c] : Q.l1[c];
}
// Fills Q for 2 <= n <= mu <= kQuadMaxMu (host; quad_tables.cpp); false otherwise.
bool make_quad_tables(int n, int mu, QuadTables* Q);

KP_INLINE double qK(const QuadTables& Q, int p, int q, int alpha, int beta) {
    return Q.K[(p * kQuadTypes + q) * kQuadMaxMu * kQuadMaxMu + alpha * kQuadMaxMu + beta];
}

// one general element: pointers into the batch arrays
struct QuadElem {
    int dim, n, mu;
    double tau;
    const double* c;   // mu^d
    const double* a;   // d x mu^d
    const double* nu;  // mu^d
    const double* g;   // 2d x mu^(d-1)
};

// ----------------------------------------------------------------- 3D terms
// term t: types (tx, ty, tz) and its group (the index of its (ty, tz) pair)
KP_INLINE void term3(int t, int* tx, int* ty, int* tz, int* grp) {
    //            mass adv_x adv_y adv_z dif_x dif_y dif_z fx- fx+ fy- fy+ fz- fz+
    const int X[13] = {0, 1, 0, 0, 2, 0, 0, 3, 4, 0, 0, 0, 0};
    const int Y[13] = {0, 0, 1, 0, 0, 2, 0, 0, 0, 3, 4, 0, 0};
    const int Z[13] = {0, 0, 0, 1, 0, 0, 2, 0, 0, 0, 0, 3, 4};
    const int G[13] = {0, 0, 1, 2, 0, 3, 4, 0, 0, 5, 6, 7, 8};
    *tx = X[t];
    *ty = Y[t];
    *tz = Z[t];
    *grp = G[t];
}
// (ty, tz) of group g
KP_INLINE void group3(int g, int* ty, int* tz) {
    const int Y[9] = {0, 1, 0, 2, 0, 3, 4, 0, 0};
    const int Z[9] = {0, 0, 1, 0, 2, 0, 0, 3, 4};
    *ty = Y[g];
    *tz = Z[g];
}
// f_t at (alpha, beta, gamma) (an index on a face's own axis is 0)
KP_INLINE double coef3(const QuadElem& el, const QuadTables& Q, int t, int al, int be, int ga) {
    const int mu = el.mu, m2 = mu * mu;
    const double* w = Q.w;
    const double tau = el.tau;
    const long p3 = ((long)al * mu + be) * mu + ga;
    switch (t) {
        case 0: return w[al] * w[be] * w[ga] * el.c[p3];
        case 1: case 2: case 3: return -tau * w[al] * w[be] * w[ga] * el.a[(long)(t - 1) * m2 * mu + p3];
        case 4: case 5: case 6: return tau * w[al] * w[be] * w[ga] * el.nu[p3];
        case 7: case 8: return tau * w[be] * w[ga] * el.g[(long)(t - 7) * m2 + be * mu + ga];
        case 9: case 10: return tau * w[al] * w[ga] * el.g[(long)(t - 7) * m2 + al * mu + ga];
        default: return tau * w[al] * w[be] * el.g[(long)(t - 7) * m2 + al * mu + be];
    }
}

// Term t's weighted coefficients in C (quad_coef_doubles layout) at (al, be, ga):
// the value coef3 returns, read with one load.  The face terms depend on two of
// the three indices (the third is the face's single point).
KP_INLINE const double* coef3_base(const double* C, int mu, int t) {
    const long m3 = (long)mu * mu * mu, m2 = (long)mu * mu;
    return t == 0 ? C : t <= 3 ? C + t * m3 : t <= 6 ? C + 4 * m3 : C + 5 * m3 + (t - 7) * m2;
}
KP_INLINE double coef3w(const double* Ct, int mu, int t, int al, int be, int ga) {
    return t <= 6 ? Ct[((long)al * mu + be) * mu + ga]
           : t <= 8 ? Ct[be * mu + ga]
           : t <= 10 ? Ct[al * mu + ga]
                     : Ct[al * mu + be];
}
// C <- the weighted coefficients of the element (the products coef3 forms, in
// its order)
template <class Team>
KP_HD void coef3_weights(const Team& tm, const QuadElem& el, const QuadTables& Q, double* C) {
    const int mu = el.mu;
    const long m3 = (long)mu * mu * mu, m2 = (long)mu * mu;
    for (long p3 = tm.tid(); p3 < m3; p3 += tm.size()) {
        const int al = (int)(p3 / m2), be = (int)((p3 / mu) % mu), ga = (int)(p3 % mu);
        C[p3] = coef3(el, Q, 0, al, be, ga);
        for (int d = 0; d < 3; ++d) C[(1 + d) * m3 + p3] = coef3(el, Q, 1 + d, al, be, ga);
        C[4 * m3 + p3] = coef3(el, Q, 4, al, be, ga);
    }
    for (long idx = tm.tid(); idx < 6 * m2; idx += tm.size()) {
        const int f = (int)(idx / m2), i = (int)((idx / mu) % mu), j = (int)(idx % mu);
        const int t = 7 + f;
        // (be, ga) for t = 7, 8; (al, ga) for 9, 10; (al, be) for 11, 12
        C[5 * m3 + idx] = t <= 8 ? coef3(el, Q, t, 0, i, j) : t <= 10 ? coef3(el, Q, t, i, 0, j) : coef3(el, Q, t, i, j, 0);
    }
    tm.sync();
}

// ----------------------------------------------------------------- 2D terms
struct Term2 {
    int tx, ty;
    const double* F;  // mu_tx x mu_ty, leading dimension ld
    int ld;
};

// the nine 2D terms of a general 2D element, with their coefficient matrices
// formed into Fbuf (9 blocks of kQuadMaxMu^2)
template <class Team>
KP_HD void terms2_of_element(const Team& tm, const QuadElem& el, const QuadTables& Q, double* Fbuf, Term2* T) {
    const int mu = el.mu;
    const int ld = kQuadMaxMu;
    const long blk = (long)ld * ld;
    //              mass adv_x adv_y dif_x dif_y fx- fx+ fy- fy+
    const int X[9] = {0, 1, 0, 2, 0, 3, 4, 0, 0};
    const int Y[9] = {0, 0, 1, 0, 2, 0, 0, 3, 4};
    for (int t = 0; t < 9; ++t) T[t] = Term2{X[t], Y[t], Fbuf + t * blk, ld};
    const double* w = Q.w;
    const double tau = el.tau;
    for (int idx = tm.tid(); idx < 9 * mu * mu; idx += tm.size()) {
        const int t = idx / (mu * mu), al = (idx / mu) % mu, be = idx % mu;
        const long p = (long)al * mu + be;
        double v;
        if (t == 0) v = w[al] * w[be] * el.c[p];
        else if (t <= 2) v = -tau * w[al] * w[be] * el.a[(long)(t - 1) * mu * mu + p];
        else if (t <= 4) v = tau * w[al] * w[be] * el.nu[p];
        else if (t <= 6) {  // x faces: a single point on x, the element's y points
            if (al > 0) continue;
            v = tau * w[be] * el.g[(long)(t - 5) * mu + be];
        } else {           // y faces: the x points, a single point on y
            if (be > 0) continue;
            v = tau * w[al] * el.g[(long)(t - 5) * mu + al];
        }
        // x faces store F[0][beta], y faces F[alpha][0]
        Fbuf[t * blk + (long)al * ld + be] = v;
    }
    tm.sync();
}

// The 3D element's weighted term coefficients (coef3 of every term, read once
// per Lanczos product instead of four loads): the mass, the three advection
// components and the diffusion (the three diffusion terms share it) as mu^3
// tensors, then the six face terms as mu^2 matrices.
KP_INLINE long quad_coef_doubles(int dim, int mu) {
    return dim == 3 ? 5L * mu * mu * mu + 6L * mu * mu : 0;
}

// Scratch of the general-element operators (team-shared): doubles needed
KP_INLINE long quad_work_doubles(int dim, int n, int mu) {
    const long M2 = (long)kQuadMaxMu * kQuadMaxMu;
    return 9 * M2 /*S*/ + 9 * M2 /*W*/ + 45 * M2 /*M*/ + 9 * M2 /*F2 or Sd*/ + 2 * kQuadMaxMu * kMaxN /*T*/ +
           2 * kQuadTypes * kQuadMaxMu /*q, Qp*/ + 5 * M2 /*R*/ + quad_coef_doubles(dim, mu) + 64 + 0 * n;
}

struct QuadScratch {
    double *S, *W, *M, *F, *T, *q, *Qp, *R;
    double* C;  // 3D: the element's weighted term coefficients (quad_coef_doubles)
};
KP_INLINE QuadScratch carve_quad(double* p) {
    const long M2 = (long)kQuadMaxMu * kQuadMaxMu;
    QuadScratch s;
    s.S = p; p += 9 * M2;
    s.W = p; p += 9 * M2;
    s.M = p; p += 45 * M2;
    s.F = p; p += 9 * M2;
    s.T = p; p += 2 * kQuadMaxMu * kMaxN;
    s.q = p; p += kQuadTypes * kQuadMaxMu;
    s.Qp = p; p += kQuadTypes * kQuadMaxMu;
    s.R = p; p += 5 * M2;
    s.C = p;
    return s;
}

// q[p][alpha] = sum_{a,c} L_p[alpha,a] x[a,c] R_p[alpha,c] for the five types;
// T: 2 mu n scratch (Phi x and dPhi x)
template <class Team>
KP_HD void quad_left(const Team& tm, const QuadTables& Q, const double* x, double* T, double* q) {
    const int n = Q.n, mu = Q.mu;
    for (int idx = tm.tid(); idx < 2 * mu * n; idx += tm.size()) {
        const int d = idx / (mu * n), al = (idx / n) % mu, c = idx % n;
        const double* L = d ? Q.dPhi : Q.Phi;
        double s = 0.0;
#pragma unroll 8
        for (int a = 0; a < n; ++a) s += L[al * n + a] * x[a * n + c];
        T[idx] = s;
    }
    double s0 = 0.0, s1 = 0.0;
    for (int t = tm.tid(); t < n * n; t += tm.size()) {
        const int a = t / n, c = t % n;
        s0 += Q.l0[a] * x[t] * Q.l0[c];
        s1 += Q.l1[a] * x[t] * Q.l1[c];
    }
    s0 = tm.sum(s0);
    s1 = tm.sum(s1);
    for (int idx = tm.tid(); idx < 3 * mu; idx += tm.size()) {
        const int p = idx / mu, al = idx % mu;
        const double* Tx = T + (p == 0 ? 0 : mu * n) + al * n;  // Phi x for PP, dPhi x for dP, dd
        const double* Rr = (p == 2 ? Q.dPhi : Q.Phi) + al * n;
        double s = 0.0;
#pragma unroll 8
        for (int c = 0; c < n; ++c) s += Tx[c] * Rr[c];
        q[p * kQuadMaxMu + al] = s;
    }
    if (tm.leader()) {
        q[3 * kQuadMaxMu] = s0;
        q[4 * kQuadMaxMu] = s1;
    }
    tm.sync();
}

// y[a,c] = sum_p sum_alpha L_p[alpha,a] Qp[p][alpha] R_p[alpha,c]
template <class Team>
KP_HD void quad_right_left(const Team& tm, const QuadTables& Q, const double* Qp, double* y) {
    const int n = Q.n, mu = Q.mu;
    for (int t = tm.tid(); t < n * n; t += tm.size()) {
        const int a = t / n, c = t % n;
        double s = 0.0;
#pragma unroll 8
        for (int al = 0; al < mu; ++al)
            s += Q.Phi[al * n + a] * Qp[al] * Q.Phi[al * n + c] +
                 Q.dPhi[al * n + a] * (Qp[kQuadMaxMu + al] * Q.Phi[al * n + c] +
                                       Qp[2 * kQuadMaxMu + al] * Q.dPhi[al * n + c]);
        s += Q.l0[a] * Qp[3 * kQuadMaxMu] * Q.l0[c] + Q.l1[a] * Qp[4 * kQuadMaxMu] * Q.l1[c];
        y[t] = s;
    }
    tm.sync();
}

// ------------------------------------------------------ 2D operator (OpQuad2)
struct OpQuad2 {
    const QuadTables* Q;
    const Term2* T;
    int nt;
    QuadScratch s;

    // S_y[beta] = sum_{t: ty = y} sum_alpha F_t[alpha, beta] q[tx][alpha]
    template <class Team>
    KP_HD void collect(const Team& tm, const double* q, double* S) const {
        const int mu = Q->mu;
        for (int idx = tm.tid(); idx < kQuadTypes * mu; idx += tm.size()) {
            const int y = idx / mu, be = idx % mu;
            double v = 0.0;
            if (be < qmu(*Q, y))
                for (int t = 0; t < nt; ++t) {
                    if (T[t].ty != y) continue;
                    const int mx = qmu(*Q, T[t].tx);
#pragma unroll 8
                    for (int al = 0; al < mx; ++al)
                        v += T[t].F[(long)al * T[t].ld + be] * q[T[t].tx * kQuadMaxMu + al];
                }
            S[y * kQuadMaxMu + be] = v;
        }
        tm.sync();
    }

    // y = R R^T x
    template <class Team>
    KP_HD void apply(const Team& tm, const double* x, double* y) const {
        const int mu = Q->mu;
        quad_left(tm, *Q, x, s.T, s.q);
        collect(tm, s.q, s.S);
        // W_y'[beta'] = sum_y sum_beta K[y][y'][beta, beta'] S_y[beta]
        for (int idx = tm.tid(); idx < kQuadTypes * mu; idx += tm.size()) {
            const int yp = idx / mu, bp = idx % mu;
            double v = 0.0;
            if (bp < qmu(*Q, yp))
                for (int yy = 0; yy < kQuadTypes; ++yy) {
                    const int my = qmu(*Q, yy);
#pragma unroll 8
                    for (int be = 0; be < my; ++be) v += qK(*Q, yy, yp, be, bp) * s.S[yy * kQuadMaxMu + be];
                }
            s.W[yp * kQuadMaxMu + bp] = v;
        }
        tm.sync();
        // Q_p[alpha] = sum_{t: tx = p} sum_beta F_t[alpha, beta] W_{ty}[beta]
        for (int idx = tm.tid(); idx < kQuadTypes * mu; idx += tm.size()) {
            const int p = idx / mu, al = idx % mu;
            double v = 0.0;
            if (al < qmu(*Q, p))
                for (int t = 0; t < nt; ++t) {
                    if (T[t].tx != p) continue;
                    const int my = qmu(*Q, T[t].ty);
#pragma unroll 8
                    for (int be = 0; be < my; ++be)
                        v += T[t].F[(long)al * T[t].ld + be] * s.W[T[t].ty * kQuadMaxMu + be];
                }
            s.Qp[p * kQuadMaxMu + al] = v;
        }
        tm.sync();
        quad_right_left(tm, *Q, s.Qp, y);
    }

    // B = sc R^T x (the right factor on the second axis' pairs)
    template <class Team>
    KP_HD void right_factor(const Team& tm, const double* x, double sc, double* B) const {
        quad_left(tm, *Q, x, s.T, s.q);
        collect(tm, s.q, s.S);
        for (int t = tm.tid(); t < kQuadTypes * kQuadMaxMu; t += tm.size()) s.Qp[t] = sc * s.S[t];
        tm.sync();
        quad_right_left(tm, *Q, s.Qp, B);
    }
};

struct RightQuad2 {
    const OpQuad2* op;
    template <class Team>
    KP_HD void operator()(const Team& tm, const double* x, double sc, double* B) const {
        op->right_factor(tm, x, sc, B);
    }
    template <class Team>
    KP_HD void forward(const Team&, const double*, double*) const {}
};

// ------------------------------------------------------ 3D operator (OpQuad3)
struct OpQuad3 {
    const QuadTables* Q;
    QuadElem el;
    QuadScratch s;

    // S_g[beta, gamma] (g < 9, leading dimension kQuadMaxMu) from q
    template <class Team>
    KP_HD void collect(const Team& tm, const double* q, double* S, double sc) const {
        const int mu = Q->mu;
        const long M2 = (long)kQuadMaxMu * kQuadMaxMu;
        for (int idx = tm.tid(); idx < kQuadGroups3 * mu * mu; idx += tm.size()) {
            const int g = idx / (mu * mu), be = (idx / mu) % mu, ga = idx % mu;
            int gy, gz;
            group3(g, &gy, &gz);
            double v = 0.0;
            if (be < qmu(*Q, gy) && ga < qmu(*Q, gz))
                for (int t = 0; t < kQuadTerms3; ++t) {
                    int tx, ty, tz, tg;
                    term3(t, &tx, &ty, &tz, &tg);
                    if (tg != g) continue;
                    const int mx = qmu(*Q, tx);
                    const double* Ct = coef3_base(s.C, mu, t);
#pragma unroll 8
                    for (int al = 0; al < mx; ++al) v += coef3w(Ct, mu, t, al, be, ga) * q[tx * kQuadMaxMu + al];
                }
            S[g * M2 + (long)be * kQuadMaxMu + ga] = sc * v;
        }
        tm.sync();
    }

    // y = R R^T x
    template <class Team>
    KP_HD void apply(const Team& tm, const double* x, double* y) const {
        const int mu = Q->mu;
        const long M2 = (long)kQuadMaxMu * kQuadMaxMu;
        quad_left(tm, *Q, x, s.T, s.q);
        collect(tm, s.q, s.S, 1.0);
        // M[g][zt][beta, gamma'] = sum_gamma S_g[beta, gamma] K[tz(g)][zt][gamma, gamma']
        for (int idx = tm.tid(); idx < kQuadGroups3 * kQuadTypes * mu * mu; idx += tm.size()) {
            const int g = idx / (kQuadTypes * mu * mu), zt = (idx / (mu * mu)) % kQuadTypes;
            const int be = (idx / mu) % mu, gp = idx % mu;
            int gy, gz;
            group3(g, &gy, &gz);
            double v = 0.0;
            if (be < qmu(*Q, gy) && gp < qmu(*Q, zt)) {
                const int mz = qmu(*Q, gz);
#pragma unroll 8
                for (int ga = 0; ga < mz; ++ga) v += s.S[g * M2 + (long)be * kQuadMaxMu + ga] * qK(*Q, gz, zt, ga, gp);
            }
            s.M[(g * kQuadTypes + zt) * M2 + (long)be * kQuadMaxMu + gp] = v;
        }
        tm.sync();
        // W_h[beta', gamma'] = sum_g sum_beta K[ty(g)][ty(h)][beta, beta'] M[g][tz(h)][beta, gamma']
        for (int idx = tm.tid(); idx < kQuadGroups3 * mu * mu; idx += tm.size()) {
            const int h = idx / (mu * mu), bp = (idx / mu) % mu, gp = idx % mu;
            int hy, hz;
            group3(h, &hy, &hz);
            double v = 0.0;
            if (bp < qmu(*Q, hy) && gp < qmu(*Q, hz))
                for (int g = 0; g < kQuadGroups3; ++g) {
                    int gy, gz;
                    group3(g, &gy, &gz);
                    const double* Mg = s.M + (g * kQuadTypes + hz) * M2;
                    const int my = qmu(*Q, gy);
#pragma unroll 8
                    for (int be = 0; be < my; ++be) v += qK(*Q, gy, hy, be, bp) * Mg[(long)be * kQuadMaxMu + gp];
                }
            s.W[h * M2 + (long)bp * kQuadMaxMu + gp] = v;
        }
        tm.sync();
        // R[p][alpha][beta] = sum_{t: tx = p} sum_gamma f_t[alpha, beta, gamma] W_{g(t)}[beta, gamma]
        for (int idx = tm.tid(); idx < kQuadTypes * mu * mu; idx += tm.size()) {
            const int p = idx / (mu * mu), al = (idx / mu) % mu, be = idx % mu;
            double v = 0.0;
            if (al < qmu(*Q, p))
                for (int t = 0; t < kQuadTerms3; ++t) {
                    int tx, ty, tz, tg;
                    term3(t, &tx, &ty, &tz, &tg);
                    if (tx != p || be >= qmu(*Q, ty)) continue;
                    const double* Wg = s.W + tg * M2 + (long)be * kQuadMaxMu;
                    const double* Ct = coef3_base(s.C, mu, t);
                    const int mz = qmu(*Q, tz);
#pragma unroll 8
                    for (int ga = 0; ga < mz; ++ga) v += coef3w(Ct, mu, t, al, be, ga) * Wg[ga];
                }
            s.R[(p * kQuadMaxMu + al) * kQuadMaxMu + be] = v;
        }
        tm.sync();
        for (int idx = tm.tid(); idx < kQuadTypes * mu; idx += tm.size()) {
            const int p = idx / mu, al = idx % mu;
            double v = 0.0;
            for (int be = 0; be < mu; ++be) v += s.R[(p * kQuadMaxMu + al) * kQuadMaxMu + be];
            s.Qp[p * kQuadMaxMu + al] = v;
        }
        tm.sync();
        quad_right_left(tm, *Q, s.Qp, y);
    }

    // the stage-1 right factor sc R^T u in factored form: Sd[g] (the groups'
    // coefficient matrices of D1) and the 2D terms of D1 pointing at them
    template <class Team>
    KP_HD void right_factor(const Team& tm, const double* u, double sc, double* Sd, Term2* T2) const {
        quad_left(tm, *Q, u, s.T, s.q);
        collect(tm, s.q, Sd, sc);
        const long M2 = (long)kQuadMaxMu * kQuadMaxMu;
        for (int g = 0; g < kQuadGroups3; ++g) {
            int gy, gz;
            group3(g, &gy, &gz);
            T2[g] = Term2{gy, gz, Sd + g * M2, kQuadMaxMu};
        }
    }
};

// Lanczos step limit of the general-element stages
KP_INLINE int quad_kmax(int n) {
    const int m = n * n;
    const int k = n + 24;
    return k < m ? k : m;
}

// Per-slot work of the general-element setup: the Lanczos work for m = n^2
// and kmax = quad_kmax(n), the three Ritz vectors, then the quad scratch
KP_INLINE long quad_setup_doubles(int dim, int n, int mu) {
    const long m = (long)n * n, k = quad_kmax(n);
    return (k + 1) * m + m + (k + 2) + 2 * (k + 1) + 2 * k + k * k + 3 * k + 3 + 8 + 2 * k + 4 + 3 * m +
           quad_work_doubles(dim, n, mu) + 64;
}
KP_INLINE SetupWork carve_quad_setup(double* p, int n, QuadScratch* qs) {
    const long m = (long)n * n, k = quad_kmax(n);
    SetupWork W = {};
    W.L.Q = p; p += (k + 1) * m;
    W.L.w = p; p += m;
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
    W.U = p; p += 3 * m;
    *qs = carve_quad(p);
    return W;
}

// Setup of one general element: factors [A1,B1,A2,B2] (2D, rank 2) or
// [A1,B1,C1,B2,C2] (3D) and singular values (2D sigma_1,2; 3D sigma_1 of
// stage 1, then sigma_1,2 of stage 2).  W: the Lanczos work of a SetupWork
// carved for (dim, n, kmax = quad_kmax(n)); qs: quad scratch.
template <class Team>
KP_HD int setup_quad_element(const Team& tm, const QuadElem& el, const QuadTables& Q, double* factors,
                             double* sigma, SetupWork& W, QuadScratch qs, Term2* T2) {
    const int n = el.n, nn = n * n;
    const int kmax = quad_kmax(n);
    int status = 0;
    for (int j = tm.tid(); j < 4; j += tm.size()) sigma[j] = 0.0;
    tm.sync();
    if (el.dim == 2) {
        terms2_of_element(tm, el, Q, qs.F, T2);
        OpQuad2 op{&Q, T2, kQuadTerms2, qs};
        RightQuad2 rq{&op};
        status |= ksvd_stage<false>(tm, op, rq, n, 2, kmax, nullptr, W, factors, 2L * nn, factors + nn, 2L * nn,
                                    n, sigma);
        return status;
    }
    coef3_weights(tm, el, Q, qs.C);
    OpQuad3 op{&Q, el, qs};
    lanczos_start(tm, W.L.Q, nn, nullptr);
    const int conv = lanczos_top(tm, op, nn, 1, kmax, 1e-14, W.L, W.U);
    status |= conv ? 0 : 1;
    canonical_sign(tm, W.U, nn, W.L.ctrl + 2);
    const double th = W.L.theta[0];
    const double s1 = sqrt(th > 0.0 ? th : 0.0);
    const double rs1 = sqrt(s1);
    if (tm.leader()) sigma[0] = s1;
    for (int i = tm.tid(); i < nn; i += tm.size()) factors[i] = rs1 * W.U[i];  // A1
    tm.sync();
    const double sc = rs1 > 0.0 ? 1.0 / rs1 : 0.0;
    // stage 2 on D1 (its coefficient matrices in qs.F)
    op.right_factor(tm, W.U, sc, qs.F, T2);
    tm.sync();
    OpQuad2 op2{&Q, T2, kQuadGroups3, qs};
    RightQuad2 rq2{&op2};
    status |= ksvd_stage<false>(tm, op2, rq2, n, 2, kmax, nullptr, W, factors + nn, 2L * nn, factors + 2 * nn,
                                2L * nn, n, sigma + 1);
    return status;
}

}  // namespace kp
