// Per-element numerical routines of the KSVD preconditioner, written against a
// team of cooperating threads (kp_common.h).  Every array argument is memory
// the whole team can read and write (LDS or global on the GPU).  A routine
// that writes shared memory ends with a team barrier before any thread reads
// what another thread wrote.
//
// Index conventions: nodal vectors are C-ordered with x slowest; matrices are
// row-major.  The rearrangement of Sec. 4.1 is taken with row-major vec: for a
// block of size (n*s) x (n*s) seen as an n x n grid of s x s sub-blocks,
//   R(A)[(a*n + a'), (K*s + K')] = A[a*s + K, a'*s + K'],
// so R(X (x) Y) = vec(X) vec(Y)^T.  2D: s = n.  3D first stage: s = n^2.
#pragma once

#include "kp_common.h"
#include "tables.h"

namespace kp {

// ============================================================ element data
// Structured form of the synthetic element block (the collocated operator of
// Sec. 3.4 with element-constant flux Jacobians):
//   A = diag(m) + sum_ax  W (x) .. (x) X_ax (x) .. (x) W,
//   m = w (x) w [(x) w] * (1 + alpha sin(pi x y [z] + phi)),
//   X_ax = tau*(beta_ax S + nu K) [+ tau*u_f l l^T for each outflow face f of
//   the axis (u_f > 0; l = l0 low face, l1 high face) with the face flag].
template <class Team>
KP_HD void record_structure(const Team& tm, const double* rec, const Tables1D& T, int dim,
                            double* mass, double* Xax) {
    const int n = T.n;
    const double alpha = rec[4], phi = rec[5], tau = rec[6], nu = rec[3];
    const bool face = rec[7] != 0.0;
    const int nd = dim == 2 ? n * n : n * n * n;
    const double pi = 3.14159265358979323846;
    for (int I = tm.tid(); I < nd; I += tm.size()) {
        int a, b, c;
        double wp, xp;
        if (dim == 2) {
            a = I / n; b = I % n;
            wp = T.w[a] * T.w[b];
            xp = T.x[a] * T.x[b];
        } else {
            a = I / (n * n); b = (I / n) % n; c = I % n;
            wp = T.w[a] * T.w[b] * T.w[c];
            xp = T.x[a] * T.x[b] * T.x[c];
        }
        mass[I] = wp * (1.0 + alpha * sin(pi * xp + phi));
    }
    for (int t = tm.tid(); t < dim * n * n; t += tm.size()) {
        const int ax = t / (n * n), ij = t % (n * n), i = ij / n, j = ij % n;
        const double beta = rec[ax];
        double v = tau * (beta * T.S[ij] + nu * T.K[ij]);
        if (face) {
            const double ulo = rec[8 + 2 * ax], uhi = rec[9 + 2 * ax];
            if (ulo > 0.0) v += tau * ulo * T.l0[i] * T.l0[j];
            if (uhi > 0.0) v += tau * uhi * T.l1[i] * T.l1[j];
        }
        Xax[t] = v;
    }
    tm.sync();
}

// One entry A[I, J] of the explicit block from its structured form.
KP_INLINE double block_entry(int dim, int n, long I, long J, const double* mass, const double* Xax,
                             const double* w) {
    if (dim == 2) {
        const int a = (int)(I / n), b = (int)(I % n), a2 = (int)(J / n), b2 = (int)(J % n);
        double v = (I == J) ? mass[I] : 0.0;
        if (b == b2) v += Xax[a * n + a2] * w[b];
        if (a == a2) v += w[a] * Xax[n * n + b * n + b2];
        return v;
    }
    const int nn = n * n;
    const int a = (int)(I / nn), b = (int)((I / n) % n), c = (int)(I % n);
    const int a2 = (int)(J / nn), b2 = (int)((J / n) % n), c2 = (int)(J % n);
    double v = (I == J) ? mass[I] : 0.0;
    if (b == b2 && c == c2) v += Xax[a * n + a2] * w[b] * w[c];
    if (a == a2 && c == c2) v += w[a] * Xax[nn + b * n + b2] * w[c];
    if (a == a2 && b == b2) v += w[a] * w[b] * Xax[2 * nn + c * n + c2];
    return v;
}

// ================================================= left Gram operators
// Each operator applies G = R(A) R(A)^T to a left vector x (length n^2, the
// flattened first Kronecker factor) and forms R(A)^T x (the second factor).

// Structured 2D block A = diag(m) + X (x) W + W (x) Y  (m: n^2, X, Y: n x n).
// R(A)^T x = diag(g) + c Y with g_k = sum_i x_ii m_ik + w_k <X,x>, c = sum_i w_i x_ii;
// G x = X t1 + diag_i( sum_k m_ik d_k + w_i t2 ), d_k = g_k + c Y_kk,
// t1 = sum_k w_k d_k, t2 = <Y, R(A)^T x>.
struct OpStruct2 {
    int n;
    const double *m, *X, *Y, *w;
    double* d;     // [n] scratch (shared)
    double* red;   // [4] scratch (shared)
    double normY2; // ||Y||_F^2

    template <class Team>
    KP_HD void transpose(const Team& tm, const double* x, double* g, double* c_out) const {
        // g[k] and c (diagonal part and multiple of Y of R(A)^T x)
        double p1 = 0.0, c = 0.0;
        for (int t = tm.tid(); t < n * n; t += tm.size()) {
            p1 += X[t] * x[t];
            if (t / n == t % n) c += w[t / n] * x[t];
        }
        p1 = tm.sum(p1);
        c = tm.sum(c);
        for (int k = tm.tid(); k < n; k += tm.size()) {
            double s = 0.0;
            #pragma unroll 8
            for (int i = 0; i < n; ++i) s += x[i * n + i] * m[i * n + k];
            g[k] = s + w[k] * p1;
        }
        *c_out = c;
        tm.sync();
    }

    template <class Team>
    KP_HD void apply(const Team& tm, const double* x, double* y) const {
        double c;
        transpose(tm, x, d, &c);  // d <- g
        double t1 = 0.0, t2 = 0.0;
        for (int k = tm.tid(); k < n; k += tm.size()) {
            t2 += Y[k * n + k] * d[k];
            t1 += w[k] * (d[k] + c * Y[k * n + k]);
        }
        t1 = tm.sum(t1);
        t2 = tm.sum(t2) + c * normY2;
        // d <- diagonal of R(A)^T x ; each thread touches only its own k
        for (int k = tm.tid(); k < n; k += tm.size()) d[k] += c * Y[k * n + k];
        tm.sync();
        for (int t = tm.tid(); t < n * n; t += tm.size()) {
            const int i = t / n, i2 = t % n;
            double v = X[t] * t1;
            if (i == i2) {
                double s = 0.0;
                #pragma unroll 8
                for (int k = 0; k < n; ++k) s += m[i * n + k] * d[k];
                v += s + w[i] * t2;
            }
            y[t] = v;
        }
        tm.sync();
    }

    // y = R(A) v for a right vector v (n x n, row-major):
    // y = diag_a( sum_K m_aK v_KK + w_a <Y, v> ) + (sum_K w_K v_KK) X
    template <class Team>
    KP_HD void forward(const Team& tm, const double* v, double* y) const {
        double py = 0.0, pw = 0.0;
        for (int t = tm.tid(); t < n * n; t += tm.size()) {
            py += Y[t] * v[t];
            if (t / n == t % n) pw += w[t / n] * v[t];
        }
        py = tm.sum(py);
        pw = tm.sum(pw);
        for (int t = tm.tid(); t < n * n; t += tm.size()) {
            const int a = t / n, a2 = t % n;
            double val = pw * X[t];
            if (a == a2) {
                double s = 0.0;
                for (int K = 0; K < n; ++K) s += m[a * n + K] * v[K * n + K];
                val += s + w[a] * py;
            }
            y[t] = val;
        }
        tm.sync();
    }

    // B = R(A)^T x as a dense n x n matrix (row-major), scaled by sc
    template <class Team>
    KP_HD void right_factor(const Team& tm, const double* x, double sc, double* B) const {
        double c;
        transpose(tm, x, d, &c);
        for (int t = tm.tid(); t < n * n; t += tm.size()) {
            const int k = t / n, k2 = t % n;
            B[t] = sc * (c * Y[t] + (k == k2 ? d[k] : 0.0));
        }
        tm.sync();
    }
};

// Structured 3D block, first stage (A ~ A1 (x) D1, s = n^2):
// A = diag(m) + X (x) W (x) W + W (x) Y (x) W + W (x) W (x) Z.
// R(A)^T x = diag(g) + c (Y (x) W + W (x) Z) with
// g_bc = sum_a x_aa m_abc + <X,x> w_b w_c, c = sum_a w_a x_aa.
struct OpStruct3 {
    int n;
    const double *m, *X, *Y, *Z, *w;
    double* d;      // [n^2] scratch
    double nrm2;    // ||Y (x) W + W (x) Z||_F^2
    // Gram form (set by precompute): with M = m as an n x n^2 matrix,
    // ww_q = w_b w_c and dg_q = Y_bb w_c + w_b Z_cc (q = b n + c),
    // G = M M^T, mv = [M ww, M dg, dg.ww, ww.ww]; then G R(A)^T x costs O(n^2)
    const double* G = nullptr;
    const double* mv = nullptr;

    // forms G (into gbuf, n^2) and mv (into vbuf, 2n + 2) on the teams that
    // can; returns whether the Gram form is in use
    template <class Team>
    KP_HD bool precompute(const Team& tm, double* gbuf, double* vbuf) {
        const int nn = n * n;
        const double* w_ = w;
        const double* Y_ = Y;
        const double* Z_ = Z;
        const int n_ = n;
        auto bf = [=](int q, int j) -> double {
            const int b = q / n_, cc = q % n_;
            return j == 0 ? w_[b] * w_[cc] : Y_[b * n_ + b] * w_[cc] + w_[b] * Z_[cc * n_ + cc];
        };
        if (!tm.gram16(m, n, nn, bf, gbuf, vbuf)) return false;
        double dgww = 0.0, ww2 = 0.0;
        for (int q = tm.tid(); q < nn; q += tm.size()) {
            const double wq = bf(q, 0), dq = bf(q, 1);
            dgww += dq * wq;
            ww2 += wq * wq;
        }
        dgww = tm.sum(dgww);
        ww2 = tm.sum(ww2);
        if (tm.leader()) {
            vbuf[2 * n] = dgww;
            vbuf[2 * n + 1] = ww2;
        }
        tm.sync();
        G = gbuf;
        mv = vbuf;
        return true;
    }

    // G R(A)^T x in the Gram form: with x_d = diag(x), p1 = <X, x>, c = w.x_d,
    //   t1 = (M ww).x_d + p1 ww.ww + c dg.ww,  t2 = (M dg).x_d + p1 dg.ww + c nrm2,
    //   y = t1 X + diag(G x_d + p1 M ww + c M dg + t2 w)
    template <class Team>
    KP_HD void apply_gram(const Team& tm, const double* x, double* y) const {
        const int nn = n * n;
        double p1 = 0.0, c = 0.0, u1 = 0.0, u2 = 0.0;
        for (int t = tm.tid(); t < nn; t += tm.size()) {
            p1 += X[t] * x[t];
            const int a = t / n;
            if (a == t % n) {
                const double xa = x[t];
                c += w[a] * xa;
                u1 += mv[a] * xa;
                u2 += mv[n + a] * xa;
            }
        }
        p1 = tm.sum(p1);
        c = tm.sum(c);
        u1 = tm.sum(u1);
        u2 = tm.sum(u2);
        const double dgww = mv[2 * n], ww2 = mv[2 * n + 1];
        const double t1 = u1 + p1 * ww2 + c * dgww;
        const double t2 = u2 + p1 * dgww + c * nrm2;
        for (int t = tm.tid(); t < nn; t += tm.size()) {
            const int a = t / n, a2 = t % n;
            double v = X[t] * t1;
            if (a == a2) {
                double s = 0.0;
                #pragma unroll 8
                for (int b = 0; b < n; ++b) s += G[a * n + b] * x[b * n + b];
                v += s + p1 * mv[a] + c * mv[n + a] + w[a] * t2;
            }
            y[t] = v;
        }
        tm.sync();
    }

    template <class Team>
    KP_HD void transpose(const Team& tm, const double* x, double* g, double* c_out) const {
        const int nn = n * n;
        double p1 = 0.0, c = 0.0;
        for (int t = tm.tid(); t < nn; t += tm.size()) {
            p1 += X[t] * x[t];
            if (t / n == t % n) c += w[t / n] * x[t];
        }
        p1 = tm.sum(p1);
        c = tm.sum(c);
        for (int q = tm.tid(); q < nn; q += tm.size()) {
            double s = 0.0;
            #pragma unroll 8
            for (int a = 0; a < n; ++a) s += x[a * n + a] * m[a * nn + q];
            g[q] = s + p1 * w[q / n] * w[q % n];
        }
        *c_out = c;
        tm.sync();
    }

    template <class Team>
    KP_HD void apply(const Team& tm, const double* x, double* y) const {
        if (G) {
            apply_gram(tm, x, y);
            return;
        }
        const int nn = n * n;
        double c;
        transpose(tm, x, d, &c);
        double t1 = 0.0, t2 = 0.0;
        for (int q = tm.tid(); q < nn; q += tm.size()) {
            const int b = q / n, cc = q % n;
            const double dg = Y[b * n + b] * w[cc] + w[b] * Z[cc * n + cc];
            t2 += dg * d[q];
            d[q] += c * dg;
            t1 += w[b] * w[cc] * d[q];
        }
        t1 = tm.sum(t1);
        t2 = tm.sum(t2) + c * nrm2;
        // s_a = sum_q m[a][q] d[q], spread over the team: C interleaved chunks
        // of q per a (partials in y), then the chunk sums in order into d[a]
        int C = tm.size() / n;
        if (C > n) C = n;
        if (C < 1) C = 1;
        for (int t = tm.tid(); t < n * C; t += tm.size()) {
            const int a = t / C, ch = t % C;
            double s = 0.0;
            for (int q = ch; q < nn; q += C) s += m[a * nn + q] * d[q];
            y[t] = s;
        }
        tm.sync();
        for (int a = tm.tid(); a < n; a += tm.size()) {
            double s = 0.0;
            for (int ch = 0; ch < C; ++ch) s += y[a * C + ch];
            d[a] = s;
        }
        tm.sync();
        for (int t = tm.tid(); t < nn; t += tm.size()) {
            const int a = t / n, a2 = t % n;
            double v = X[t] * t1;
            if (a == a2) v += d[a] + w[a] * t2;
            y[t] = v;
        }
        tm.sync();
    }

    // D1 = sc * R(A)^T x in structured 2D form: mass' = sc*g, X' = sc*c*Y, Y' = sc*c*Z
    template <class Team>
    KP_HD void right_factor(const Team& tm, const double* x, double sc, double* m2, double* X2,
                            double* Y2) const {
        double c;
        transpose(tm, x, m2, &c);
        for (int q = tm.tid(); q < n * n; q += tm.size()) {
            m2[q] *= sc;
            X2[q] = sc * c * Y[q];
            Y2[q] = sc * c * Z[q];
        }
        tm.sync();
    }
};

// Explicit block, Gram held in memory: G (msz x msz).
struct OpGram {
    int msz;
    const double* G;
    template <class Team>
    KP_HD void apply(const Team& tm, const double* x, double* y) const {
        for (int i = tm.tid(); i < msz; i += tm.size()) {
            double s = 0.0;
#pragma unroll 8
            for (int j = 0; j < msz; ++j) s += G[(long)i * msz + j] * x[j];
            y[i] = s;
        }
        tm.sync();
    }
};

// Explicit block streamed from memory on every product (one pass over the
// block per application of G).  Block is (n*s) x (n*s); left vectors n^2.
// For every K the rows {a*s + K} hold R(A)[:, K*s + K'] for all K', so
// Y[K, :] = x^T R(A)[:, K*s + :] and G x += R(A)[:, K*s + :] Y[K, :]^T.
struct OpStream {
    int n, s;
    const double* A;
    double* yk;   // [s^2] scratch (apply only)
    // y = R(A) R(A)^T x in two passes over the block: z = R(A)^T x (s^2
    // entries, one per thread at a time), then y = R(A) z (one per thread);
    // each sum's terms eight at a time so that their loads are in flight
    // together
    template <class Team>
    KP_HD void apply(const Team& tm, const double* x, double* y) const {
        const int m = n * n;
        const long N = (long)n * s;
        const long ss = (long)s * s;
        for (long q = tm.tid(); q < ss; q += tm.size()) {
            const int K = (int)(q / s), K2 = (int)(q % s);
            // yk[K s + K'] = sum_{a,a'} x[a n + a'] A[(a s + K) N + a' s + K']
            double acc = 0.0;
#pragma unroll 8
            for (int t = 0; t < m; ++t) {
                const int a = t / n, a2 = t % n;
                acc += x[t] * A[((long)a * s + K) * N + (long)a2 * s + K2];
            }
            yk[q] = acc;
        }
        tm.sync();
        for (int t = tm.tid(); t < m; t += tm.size()) {
            const int a = t / n, a2 = t % n;
            double acc = 0.0;
            for (int K = 0; K < s; ++K) {
                const double* row = A + ((long)a * s + K) * N + (long)a2 * s;
#pragma unroll 8
                for (int K2 = 0; K2 < s; ++K2) acc += row[K2] * yk[(long)K * s + K2];
            }
            y[t] = acc;
        }
        tm.sync();
    }
    // y = R(A) v for a right vector v (s x s): y[a n + a2] = sum_{K,K2} A[a s + K, a2 s + K2] v[K s + K2]
    template <class Team>
    KP_HD void forward(const Team& tm, const double* v, double* y) const {
        const int m = n * n;
        const long N = (long)n * s;
        for (int t = tm.tid(); t < m; t += tm.size()) {
            const int a = t / n, a2 = t % n;
            double acc = 0.0;
            for (int K = 0; K < s; ++K) {
                const double* row = A + ((long)a * s + K) * N + (long)a2 * s;
#pragma unroll 8
                for (int K2 = 0; K2 < s; ++K2) acc += row[K2] * v[(long)K * s + K2];
            }
            y[t] = acc;
        }
        tm.sync();
    }

    // B = sc * R(A)^T x, an s x s matrix
    template <class Team>
    KP_HD void right_factor(const Team& tm, const double* x, double sc, double* B) const {
        const int m = n * n;
        const long N = (long)n * s;
        for (long q = tm.tid(); q < (long)s * s; q += tm.size()) {
            const int K = (int)(q / s), K2 = (int)(q % s);
            double acc = 0.0;
#pragma unroll 8
            for (int t = 0; t < m; ++t) {
                const int a = t / n, a2 = t % n;
                acc += x[t] * A[((long)a * s + K) * N + (long)a2 * s + K2];
            }
            B[q] = sc * acc;
        }
        tm.sync();
    }
};

// Gram of an explicit block: G[(a,a'),(b,b')] = sum_{K,K'} A[aS+K, a'S+K'] A[bS+K, b'S+K'].
template <class Team>
KP_HD void explicit_gram(const Team& tm, int n, int s, const double* A, double* G) {
    const int m = n * n;
    const long N = (long)n * s;
    for (int idx = tm.tid(); idx < m * m; idx += tm.size()) {
        const int p = idx / m, q = idx % m;
        if (q < p) continue;
        const int a = p / n, a2 = p % n, b = q / n, b2 = q % n;
        double acc = 0.0;
        for (int K = 0; K < s; ++K) {
            const double* ra = A + ((long)a * s + K) * N + (long)a2 * s;
            const double* rb = A + ((long)b * s + K) * N + (long)b2 * s;
#pragma unroll 8
            for (int K2 = 0; K2 < s; ++K2) acc += ra[K2] * rb[K2];
        }
        G[(long)p * m + q] = acc;
        G[(long)q * m + p] = acc;
    }
    tm.sync();
}

// ============================================ symmetric tridiagonal eigen
// Implicit QL with Wilkinson-type shifts on T = tridiag(e, d, e).
// d[0..k): diagonal (overwritten by eigenvalues), e[0..k-1): off-diagonal
// (destroyed, needs k entries), Z[i*k + j]: component i of eigenvector j.
// Returns false if an eigenvalue needed more than 60 sweeps.
KP_INLINE bool tridiag_eig(int k, double* d, double* e, double* Z) {
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) Z[i * k + j] = (i == j) ? 1.0 : 0.0;
    if (k == 1) return true;
    e[k - 1] = 0.0;
    const double eps = 2.220446049250313e-16;
    for (int l = 0; l < k; ++l) {
        int iter = 0;
        while (true) {
            int mm = l;
            for (; mm < k - 1; ++mm) {
                const double dd = fabs(d[mm]) + fabs(d[mm + 1]);
                if (fabs(e[mm]) <= eps * dd) break;
            }
            if (mm == l) break;
            if (++iter > 60) return false;
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = d[mm] - d[l] + e[l] / (g + (g >= 0.0 ? fabs(r) : -fabs(r)));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = mm - 1;
            bool early = false;
            for (; i >= l; --i) {
                double f = s * e[i], b = c * e[i];
                r = hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[mm] = 0.0;
                    early = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                for (int q = 0; q < k; ++q) {
                    f = Z[q * k + i + 1];
                    Z[q * k + i + 1] = s * Z[q * k + i] + c * f;
                    Z[q * k + i] = c * Z[q * k + i] - s * f;
                }
            }
            if (early) continue;
            d[l] -= p;
            e[l] = g;
            e[mm] = 0.0;
        }
    }
    return true;
}

// The same QL iteration with the eigenvector updates spread over a team:
// the leader runs each sweep (the scalar recurrence, identical arithmetic)
// and records its rotations in rot; then every thread applies the sweep's
// rotations to its own rows of Z.  Results equal tridiag_eig's.
// rot: 2 k doubles; qc: 8 ints of shared control state.
template <class Team>
KP_HD bool tridiag_eig_team(const Team& tm, int k, double* d, double* e, double* Z, double* rot, int* qc) {
    for (int t = tm.tid(); t < k * k; t += tm.size()) Z[t] = (t / k == t % k) ? 1.0 : 0.0;
    if (k == 1) {
        tm.sync();
        return true;
    }
    if (tm.leader()) {
        e[k - 1] = 0.0;
        qc[0] = 0;  // l
        qc[1] = 0;  // iterations at this l
    }
    tm.sync();
    const double eps = 2.220446049250313e-16;
    while (true) {
        if (tm.leader()) {
            int l = qc[0], iter = qc[1];
            int status = 0, mm_out = 0, ilow = 0;
            while (true) {
                if (l >= k) {
                    status = 1;
                    break;
                }
                int mm = l;
                for (; mm < k - 1; ++mm) {
                    const double dd = fabs(d[mm]) + fabs(d[mm + 1]);
                    if (fabs(e[mm]) <= eps * dd) break;
                }
                if (mm == l) {
                    ++l;
                    iter = 0;
                    continue;
                }
                if (++iter > 60) {
                    status = 2;
                    break;
                }
                double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
                double r = hypot(g, 1.0);
                g = d[mm] - d[l] + e[l] / (g + (g >= 0.0 ? fabs(r) : -fabs(r)));
                double s = 1.0, c = 1.0, p = 0.0;
                int i = mm - 1;
                bool early = false;
                for (; i >= l; --i) {
                    const double f = s * e[i], b = c * e[i];
                    r = hypot(f, g);
                    e[i + 1] = r;
                    if (r == 0.0) {
                        d[i + 1] -= p;
                        e[mm] = 0.0;
                        early = true;
                        break;
                    }
                    s = f / r;
                    c = g / r;
                    g = d[i + 1] - p;
                    r = (d[i] - g) * s + 2.0 * c * b;
                    p = s * r;
                    d[i + 1] = g + p;
                    g = c * r - b;
                    rot[2 * i] = s;
                    rot[2 * i + 1] = c;
                }
                if (!early) {
                    d[l] -= p;
                    e[l] = g;
                    e[mm] = 0.0;
                }
                mm_out = mm;
                ilow = early ? i + 1 : l;
                break;
            }
            qc[0] = l;
            qc[1] = iter;
            qc[2] = status;
            qc[3] = mm_out;
            qc[4] = ilow;
        }
        tm.sync();
        const int status = qc[2];
        if (status != 0) return status == 1;
        const int mm = qc[3], ilow = qc[4];
        for (int q = tm.tid(); q < k; q += tm.size()) {
            double* zr = Z + q * k;
            for (int i = mm - 1; i >= ilow; --i) {
                const double sn = rot[2 * i], cs = rot[2 * i + 1];
                const double f = zr[i + 1];
                zr[i + 1] = sn * zr[i] + cs * f;
                zr[i] = cs * zr[i] - sn * f;
            }
        }
        tm.sync();
    }
}

// ==================================================== Lanczos (Alg. 2)
// Top-r eigenpairs of G = R(A) R(A)^T by symmetric Lanczos with full
// reorthogonalisation (classical Gram-Schmidt, applied twice).  Its Krylov
// basis is that of the Golub-Kahan bidiagonalisation of Alg. 2 started from
// the same vector, and its tridiagonal matrix equals B^T B for the
// bidiagonal B of Alg. 2, so the Ritz values are the squared Ritz singular
// values; the right vectors follow as R(A)^T u / sigma.  One product with G
// needs one pass over R(A) instead of the two of Alg. 2.
struct LanczosWork {
    double* Q;      // (kmax+1) x m basis; Q[0..m) holds the start vector on entry
    double* w;      // m
    double* qv;     // m: a copy of the newest basis vector in fast memory, or null
    double* h;      // kmax + 2
    double* alpha;  // kmax + 1
    double* beta;   // kmax + 1
    double* d;      // kmax   (leader scratch)
    double* e;      // kmax
    double* Z;      // kmax*kmax
    double* sel;    // r * kmax selected eigenvectors of T
    double* theta;  // r
    int* ctrl;      // 8 ints: [0] converged flag, [1] steps, [4..4+r) selected Ritz indices
    double* rot;    // 2 kmax: rotations of one QL sweep
    int* qc;        // 8 ints: QL control state
};

template <class Team, class Op>
KP_HD int lanczos_top(const Team& tm, const Op& op, int m, int r, int kmax, double tol,
                      const LanczosWork& L, double* U /* r x m */, bool full = false) {
    // full: build the basis until it is invariant (beta <= 1e-14 of the scale)
    // or kmax steps, for the two-sided refinement; the Ritz test is skipped
    double* Q = L.Q;
    // normalise the start vector
    double p = 0.0;
    for (int i = tm.tid(); i < m; i += tm.size()) p += Q[i] * Q[i];
    double nrm = sqrt(tm.sum(p));
    if (!(nrm > 0.0)) {
        for (int i = tm.tid(); i < m; i += tm.size()) Q[i] = 1.0;
        nrm = sqrt((double)m);
    }
    for (int i = tm.tid(); i < m; i += tm.size()) {
        Q[i] /= nrm;
        if (L.qv) L.qv[i] = Q[i];
    }
    tm.sync();
    double scale = 0.0;
    int steps = 0;
    bool converged = false;
    for (int k = 0; k < kmax; ++k) {
        const double* qk = L.qv ? L.qv : Q + (long)k * m;
        op.apply(tm, qk, L.w);
        double aco = 0.0;
        for (int pass = 0; pass < 2; ++pass) {
            tm.dots(Q, m, k + 1, L.w, m, L.h);
            for (int i = tm.tid(); i < m; i += tm.size()) {
                double s = L.w[i];
                int j = 0;
                for (; j + 8 <= k + 1; j += 8) {  // eight basis loads in flight, the same order
                    double qv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) qv[u] = Q[(long)(j + u) * m + i];
#pragma unroll
                    for (int u = 0; u < 8; ++u) s -= L.h[j + u] * qv[u];
                }
                if (j <= k) {  // the last k + 1 - j < 8 vectors: loads in flight together (clamped rows unused)
                    double qv[7];
#pragma unroll
                    for (int u = 0; u < 7; ++u) qv[u] = Q[(long)(j + u <= k ? j + u : k) * m + i];
#pragma unroll
                    for (int u = 0; u < 7; ++u)
                        if (j + u <= k) s -= L.h[j + u] * qv[u];
                }
                L.w[i] = s;
            }
            aco += L.h[k];
            tm.sync();
        }
        double b2 = 0.0;
        for (int i = tm.tid(); i < m; i += tm.size()) b2 += L.w[i] * L.w[i];
        const double b = sqrt(tm.sum(b2));
        if (tm.leader()) {
            L.alpha[k] = aco;
            L.beta[k] = b;
        }
        scale = fmax(scale, fabs(aco) + b);
        steps = k + 1;
        const bool invariant = b <= 1e-14 * scale;
        const bool check = full ? (steps == kmax || steps == m || invariant)
                                : (steps >= r + 1 && ((steps % 4) == 0 || b <= 1e-10 * scale)) ||
                                      steps == kmax || steps == m || b == 0.0;
        if (check) {
            tm.sync();
            if (tm.leader()) {
                for (int i = 0; i < steps; ++i) {
                    L.d[i] = L.alpha[i];
                    L.e[i] = (i + 1 < steps) ? L.beta[i] : 0.0;
                }
            }
            tm.sync();
            const bool ok = tridiag_eig_team(tm, steps, L.d, L.e, L.Z, L.rot, L.qc);
            if (tm.leader()) {
                // select the r largest Ritz values (descending)
                int rr = r < steps ? r : steps;
                bool conv = ok;
                double thmax = 0.0;
                for (int i = 0; i < steps; ++i) thmax = fmax(thmax, L.d[i]);
                for (int j = 0; j < r; ++j) {
                    int best = -1;
                    for (int i = 0; i < steps; ++i) {
                        bool used = false;
                        for (int q = 0; q < j && q < rr; ++q)
                            if (L.ctrl[4 + q] == i) used = true;
                        if (used) continue;
                        if (best < 0 || L.d[i] > L.d[best]) best = i;
                    }
                    if (j < rr) {
                        L.ctrl[4 + j] = best;
                        L.theta[j] = L.d[best];
                        for (int t = 0; t < steps; ++t) L.sel[j * kmax + t] = L.Z[t * steps + best];
                        const double res = fabs(b * L.Z[(steps - 1) * steps + best]);
                        if (res > tol * thmax) conv = false;
                    } else {
                        L.theta[j] = 0.0;
                        for (int t = 0; t < steps; ++t) L.sel[j * kmax + t] = 0.0;
                        conv = false;
                    }
                }
                if (b == 0.0 && rr == r) conv = ok;
                if (full) conv = ok;
                L.ctrl[0] = conv ? 1 : 0;
            }
            tm.sync();
            if (L.ctrl[0]) {
                converged = true;
                break;
            }
        }
        if (b == 0.0 || steps == m) break;
        double* qn = Q + (long)(k + 1) * m;
        for (int i = tm.tid(); i < m; i += tm.size()) {
            const double v = L.w[i] / b;
            qn[i] = v;
            if (L.qv) L.qv[i] = v;
        }
        tm.sync();
    }
    // Ritz vectors u_j = Q sel_j (basis loads eight at a time, the same order)
    for (long t = tm.tid(); t < (long)r * m; t += tm.size()) {
        const int j = (int)(t / m), i = (int)(t % m);
        double s = 0.0;
        for (int q0 = 0; q0 < steps; q0 += 8) {
            double qv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) qv[u] = Q[(long)(q0 + u < steps ? q0 + u : steps - 1) * m + i];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (q0 + u < steps) s += L.sel[j * kmax + q0 + u] * qv[u];
        }
        U[t] = s;
    }
    tm.sync();
    if (tm.leader()) L.ctrl[1] = steps;
    tm.sync();
    return converged ? 1 : 0;
}

// flip u (and the matching right factor) so that its largest |entry| is
// positive (lowest index on ties); returns the sign applied
template <class Team>
KP_HD double canonical_sign(const Team& tm, double* u, int m, int* ctrl_slot) {
    (void)ctrl_slot;
    const int best = tm.argmax_abs(u, 1, 0, m);
    const double sg = u[best] < 0.0 ? -1.0 : 1.0;
    tm.sync();
    for (int i = tm.tid(); i < m; i += tm.size()) u[i] *= sg;
    tm.sync();
    return sg;
}

// =============================================== small dense linear algebra
// n x n row-major; team-parallel over rows/columns.

// C = A B  (C must not alias A or B)
template <class Team>
KP_HD void mm(const Team& tm, int n, const double* A, const double* B, double* C) {
    for (int t = tm.tid(); t < n * n; t += tm.size()) {
        const int i = t / n, j = t % n;
        double s = 0.0;
        #pragma unroll 8
        for (int k = 0; k < n; ++k) s += A[i * n + k] * B[k * n + j];
        C[t] = s;
    }
    tm.sync();
}
// C = A^T B
template <class Team>
KP_HD void mtm(const Team& tm, int n, const double* A, const double* B, double* C) {
    for (int t = tm.tid(); t < n * n; t += tm.size()) {
        const int i = t / n, j = t % n;
        double s = 0.0;
        #pragma unroll 8
        for (int k = 0; k < n; ++k) s += A[k * n + i] * B[k * n + j];
        C[t] = s;
    }
    tm.sync();
}

// 1-norm (largest column sum of magnitudes), returned to every thread
template <class Team>
KP_HD double norm1(const Team& tm, int n, const double* M, double* sh) {
    (void)sh;
    double mx = 0.0;
    for (int j = tm.tid(); j < n; j += tm.size()) {
        double c = 0.0;
        for (int i = 0; i < n; ++i) c += fabs(M[i * n + j]);
        mx = c > mx ? c : mx;
    }
    return tm.max(mx);
}

// Ainv = A^{-1} by Gauss-Jordan elimination with partial pivoting on the pair
// [A | I]; A is destroyed.  mult: n doubles of shared scratch; piv unused
// (kept for the call sites).  Returns false on a zero pivot.
template <class Team>
KP_HD bool invert(const Team& tm, int n, double* A, double* Ainv, int* piv, double* mult) {
    (void)piv;
    bool ok = true;
    for (int t = tm.tid(); t < n * n; t += tm.size()) Ainv[t] = (t / n == t % n) ? 1.0 : 0.0;
    tm.sync();
    for (int k = 0; k < n; ++k) {
        const int p = tm.argmax_abs(A + k, n, k, n);
        if (p != k) {
            for (int j = tm.tid(); j < 2 * n; j += tm.size()) {
                double* M = j < n ? A : Ainv;
                const int jj = j < n ? j : j - n;
                const double t = M[k * n + jj];
                M[k * n + jj] = M[p * n + jj];
                M[p * n + jj] = t;
            }
            tm.sync();
        }
        const double pv = A[k * n + k];
        if (pv == 0.0) {
            ok = false;
            continue;
        }
        // multipliers of column k (applied to the scaled pivot row), then scale
        // row k and eliminate every other row
        for (int i = tm.tid(); i < n; i += tm.size()) mult[i] = (i == k) ? 0.0 : A[i * n + k];
        tm.sync();
        const double inv = 1.0 / pv;
        for (int j = tm.tid(); j < 2 * n; j += tm.size()) {
            double* M = j < n ? A : Ainv;
            const int jj = j < n ? j : j - n;
            M[k * n + jj] *= inv;
        }
        tm.sync();
        for (int t = tm.tid(); t < 2 * n * n; t += tm.size()) {
            const int i = t / (2 * n), j = t % (2 * n);
            if (i == k) continue;
            double* M = j < n ? A : Ainv;
            const int jj = j < n ? j : j - n;
            M[i * n + jj] -= mult[i] * M[k * n + jj];
        }
        tm.sync();
    }
    return ok;
}

// ---------------------------------------------------------- real Schur form
// H <- Q^T H Q upper quasi-triangular with standardised 2x2 blocks (equal
// diagonal entries, off-diagonal product < 0, i.e. a complex-conjugate pair);
// real eigenvalue pairs are split into 1x1 blocks.  Householder reduction to
// Hessenberg form, then Francis double-shift QR steps with deflation.
// Returns false if the iteration limit was reached.

// apply the reflector I - tau v v^T (v of length len, v[0] = 1 implied by
// storage) to rows r0..r0+len-1 of H for columns c0..c1, and to columns
// r0..r0+len-1 for rows 0..rend, and to the same columns of Q.
template <class Team>
KP_HD void reflect(const Team& tm, int n, double* H, double* Q, const double* v, int len,
                   double tau, int r0, int c0, int rend) {
    if (tau == 0.0) return;
    for (int c = c0 + tm.tid(); c < n; c += tm.size()) {
        double s = 0.0;
        for (int i = 0; i < len; ++i) s += v[i] * H[(r0 + i) * n + c];
        s *= tau;
        for (int i = 0; i < len; ++i) H[(r0 + i) * n + c] -= s * v[i];
    }
    tm.sync();
    for (int r = tm.tid(); r <= rend; r += tm.size()) {
        double s = 0.0;
        for (int i = 0; i < len; ++i) s += H[r * n + r0 + i] * v[i];
        s *= tau;
        for (int i = 0; i < len; ++i) H[r * n + r0 + i] -= s * v[i];
    }
    for (int r = tm.tid(); r < n; r += tm.size()) {
        double s = 0.0;
        for (int i = 0; i < len; ++i) s += Q[r * n + r0 + i] * v[i];
        s *= tau;
        for (int i = 0; i < len; ++i) Q[r * n + r0 + i] -= s * v[i];
    }
    tm.sync();
}

// Householder vector for x (len <= 3): (I - tau v v^T) x = beta e1, v[0] = 1.
KP_INLINE void house(const double* x, int len, double* v, double* tau) {
    double sig = 0.0;
    for (int i = 1; i < len; ++i) sig += x[i] * x[i];
    v[0] = 1.0;
    for (int i = 1; i < len; ++i) v[i] = x[i];
    if (sig == 0.0) {
        *tau = 0.0;
        return;
    }
    const double mu = sqrt(x[0] * x[0] + sig);
    const double v0 = x[0] <= 0.0 ? x[0] - mu : -sig / (x[0] + mu);
    *tau = 2.0 * v0 * v0 / (sig + v0 * v0);
    for (int i = 1; i < len; ++i) v[i] = x[i] / v0;
}

// rotation of rows/columns i, i+1 by G = [[c, -s], [s, c]]: H <- G^T H G, Q <- Q G
template <class Team>
KP_HD void rotate(const Team& tm, int n, double* H, double* Q, int i, double c, double s) {
    // columns left of i and rows below i+1 are zero in the quasi-triangle
    for (int j = i + tm.tid(); j < n; j += tm.size()) {
        const double a = H[i * n + j], b = H[(i + 1) * n + j];
        H[i * n + j] = c * a + s * b;
        H[(i + 1) * n + j] = -s * a + c * b;
    }
    tm.sync();
    for (int r = tm.tid(); r < n; r += tm.size()) {
        if (r <= i + 1) {
            const double a = H[r * n + i], b = H[r * n + i + 1];
            H[r * n + i] = c * a + s * b;
            H[r * n + i + 1] = -s * a + c * b;
        }
        const double qa = Q[r * n + i], qb = Q[r * n + i + 1];
        Q[r * n + i] = c * qa + s * qb;
        Q[r * n + i + 1] = -s * qa + c * qb;
    }
    tm.sync();
}

// standardise the 2x2 diagonal block at (i, i+1): a real-eigenvalue block is
// rotated to upper triangular form, a complex pair to equal diagonal entries
template <class Team>
KP_HD void standardise2(const Team& tm, int n, double* H, double* Q, int i, double* sh) {
    for (int pass = 0; pass < 2; ++pass) {
        if (tm.leader()) {
            const double a = H[i * n + i], b = H[i * n + i + 1], c = H[(i + 1) * n + i],
                         d = H[(i + 1) * n + i + 1];
            double cs = 1.0, sn = 0.0;
            int kind = 0;  // 0 nothing, 1 triangularise, 2 equalise diagonal
            if (c != 0.0) {
                const double p = 0.5 * (a - d);
                const double disc = p * p + b * c;
                if (disc >= 0.0 || pass == 1) {
                    const double rt = sqrt(fmax(disc, 0.0));
                    const double lam = 0.5 * (a + d) + (p >= 0.0 ? rt : -rt);
                    double x0 = lam - d, x1 = c;
                    const double u0 = b, u1 = lam - a;
                    if (fabs(u0) + fabs(u1) > fabs(x0) + fabs(x1)) { x0 = u0; x1 = u1; }
                    const double nr = hypot(x0, x1);
                    if (nr > 0.0) { cs = x0 / nr; sn = x1 / nr; kind = 1; }
                } else {
                    const double th = 0.5 * atan2(d - a, b + c);
                    cs = cos(th);
                    sn = sin(th);
                    kind = 2;
                }
            }
            sh[0] = cs; sh[1] = sn; sh[2] = (double)kind;
        }
        tm.sync();
        const double cs = sh[0], sn = sh[1];
        const int kind = (int)sh[2];
        tm.sync();
        if (kind == 0) return;
        rotate(tm, n, H, Q, i, cs, sn);
        int again = 0;
        if (tm.leader()) {
            if (kind == 1) {
                H[(i + 1) * n + i] = 0.0;
            } else {
                const double avg = 0.5 * (H[i * n + i] + H[(i + 1) * n + i + 1]);
                H[i * n + i] = avg;
                H[(i + 1) * n + i + 1] = avg;
                // a complex pair has off-diagonals of opposite sign; if rounding
                // says otherwise the block is split as a real pair
                again = (H[i * n + i + 1] * H[(i + 1) * n + i] >= 0.0) ? 1 : 0;
            }
            sh[3] = (double)again;
        }
        tm.sync();
        if (sh[3] == 0.0) return;
        tm.sync();
    }
}

template <class Team>
KP_HD bool real_schur(const Team& tm, int n, double* H, double* Q, double* sh /*[kMaxN+8] shared*/) {
    for (int t = tm.tid(); t < n * n; t += tm.size()) Q[t] = (t / n == t % n) ? 1.0 : 0.0;
    tm.sync();
    // Hessenberg reduction
    for (int k = 0; k + 2 < n; ++k) {
        const int len = n - k - 1;
        if (tm.leader()) {
            double sig = 0.0;
            const double x0 = H[(k + 1) * n + k];
            for (int i = 1; i < len; ++i) sig += H[(k + 1 + i) * n + k] * H[(k + 1 + i) * n + k];
            double tau = 0.0, v0 = 1.0;
            if (sig != 0.0) {
                const double mu = sqrt(x0 * x0 + sig);
                v0 = x0 <= 0.0 ? x0 - mu : -sig / (x0 + mu);
                tau = 2.0 * v0 * v0 / (sig + v0 * v0);
            }
            sh[0] = tau;
            sh[1] = v0;
        }
        tm.sync();
        const double tau = sh[0], v0 = sh[1];
        if (tau == 0.0) {
            tm.sync();
            continue;
        }
        // build v in a scratch column: use sh[2..] (len <= kMaxN-1)
        for (int i = tm.tid(); i < len; i += tm.size())
            sh[2 + i] = (i == 0) ? 1.0 : H[(k + 1 + i) * n + k] / v0;
        tm.sync();
        reflect(tm, n, H, Q, sh + 2, len, tau, k + 1, k, n - 1);
        for (int i = 2 + tm.tid(); i < n - k; i += tm.size()) H[(k + i) * n + k] = 0.0;
        tm.sync();
    }
    // Francis QR
    const double eps = 2.220446049250313e-16;
    double hnorm = 0.0;
    for (int t = tm.tid(); t < n * n; t += tm.size()) hnorm = fmax(hnorm, fabs(H[t]));
    hnorm = tm.max(hnorm);
    int hi = n - 1, iter = 0, total = 0;
    bool ok = true;
    while (hi >= 0) {
        int l = hi;
        while (l > 0) {
            double s = fabs(H[(l - 1) * n + l - 1]) + fabs(H[l * n + l]);
            if (s == 0.0) s = hnorm;
            if (fabs(H[l * n + l - 1]) <= eps * s) break;
            --l;
        }
        tm.sync();
        if (l > 0 && tm.leader()) H[l * n + l - 1] = 0.0;
        tm.sync();
        if (l == hi) {
            --hi;
            iter = 0;
            continue;
        }
        if (l == hi - 1) {
            standardise2(tm, n, H, Q, hi - 1, sh);
            hi -= 2;
            iter = 0;
            continue;
        }
        ++iter;
        if (++total > 40 * n) {
            ok = false;
            break;
        }
        double s, t;
        if (iter % 11 == 10) {
            const double ss = fabs(H[hi * n + hi - 1]) + fabs(H[(hi - 1) * n + hi - 2]);
            s = 1.5 * ss;
            t = ss * ss;
        } else {
            s = H[(hi - 1) * n + hi - 1] + H[hi * n + hi];
            t = H[(hi - 1) * n + hi - 1] * H[hi * n + hi] - H[(hi - 1) * n + hi] * H[hi * n + hi - 1];
        }
        const int mw = hi - l + 1;
        double x = H[l * n + l] * H[l * n + l] + H[l * n + l + 1] * H[(l + 1) * n + l] -
                   s * H[l * n + l] + t;
        double y = H[(l + 1) * n + l] * (H[l * n + l] + H[(l + 1) * n + l + 1] - s);
        double z = H[(l + 1) * n + l] * H[(l + 2) * n + l + 1];
        for (int k = 0; k + 3 <= mw; ++k) {
            double xv[3] = {x, y, z}, v[3], tau;
            house(xv, 3, v, &tau);
            tm.sync();
            const int r0 = l + k;
            const int c0 = l + (k > 0 ? k - 1 : 0);
            const int rend = l + (k + 3 < mw - 1 ? k + 3 : mw - 1);
            reflect(tm, n, H, Q, v, 3, tau, r0, c0, rend);
            if (k > 0 && tm.leader()) {
                H[(r0 + 1) * n + r0 - 1] = 0.0;
                H[(r0 + 2) * n + r0 - 1] = 0.0;
            }
            tm.sync();
            x = H[(r0 + 1) * n + r0];
            y = H[(r0 + 2) * n + r0];
            if (k + 3 < mw) z = H[(r0 + 3) * n + r0];
        }
        {
            double xv[2] = {x, y}, v[2], tau;
            house(xv, 2, v, &tau);
            tm.sync();
            reflect(tm, n, H, Q, v, 2, tau, hi - 1, hi - 2, hi);
            if (tm.leader()) H[hi * n + hi - 2] = 0.0;
            tm.sync();
        }
    }
    // clean below the quasi-triangle
    for (int t = tm.tid(); t < n * n; t += tm.size()) {
        const int i = t / n, j = t % n;
        if (i > j + 1) H[t] = 0.0;
    }
    tm.sync();
    return ok;
}

// ================================================== apply tables
// Layout of one element's tables (entries of n x n matrices, row-major):
//   [0] L0 [1] L1 [2] L2 [3] R0 [4] R1 [5] T1 [6] T2 [7 .. 7+n) N_j
// 2D (P = A1 (x) B1 + A2 (x) B2): L0 = Q1^T A2^{-1}, L1 = Q2^T B1^{-1}, L2 = 0,
//   R0 = Q1, R1 = Q2, with A2^{-1}A1 = Q1 T1 Q1^T, B1^{-1}B2 = Q2 T2 Q2^T.
// 3D (P = A1 (x) B1 (x) C1 + A1 (x) B2 (x) C2): L0 = A1^{-1}, L1 = Q1^T B2^{-1},
//   L2 = Q2^T C1^{-1}, R0 = Q1, R1 = Q2, B2^{-1}B1 = Q1 T1 Q1^T, C1^{-1}C2 = Q2 T2 Q2^T.
// 2D rank 1 is expressed in the same form with T1 = T2 = I/2, Q = I.
// The quasi-triangular solve of T1 Y + Y T2^T = F sweeps the columns j of Y
// from last to first.  A 1x1 block of T2 gives y_j = N_j g_j with
// N_j = (T1 + T2[j,j] I)^{-1}.  A standardised 2x2 block at (j-1, j) with
// diagonal p and off-diagonals q = T2[j-1,j], s = T2[j,j-1] gives, for
// M = T1 + p I:  (M^2 - q s I) y_{j-1} = M g_{j-1} - q g_j and
//                (M^2 - q s I) y_j     = M g_j - s g_{j-1};
// N_{j-1} = N_j = (M^2 - q s I)^{-1}.  kinds[j]: 0 single, 1 first of a pair,
// 2 second of a pair.
constexpr int kTabFixed = 7;
KP_INLINE long tab_entries(int n) { return (long)(kTabFixed + n) * n * n; }

// The formation runs in three phases (separate kernels on the GPU, so that
// the Schur phase can run at high occupancy):
//   prepare: pair rotation, inverses of the factors to invert (stored in the
//            L slots), the matrices C1, C2 to triangularise (stored in the
//            first two N slots);
//   schur:   T_i, Q_i of C_i (into the T and R slots);
//   finish:  L = Q^T inverse (2D: L0, L1; 3D: L1, L2), block kinds of T2, N_j.

// prepare.  Work: >= 10 n^2 doubles.  F: factors (2D rank r: A1,B1,A2,B2,..;
// 3D: A1,B1,C1,B2,C2).  tab: the 7 + n matrices of the element.
template <class Team>
KP_HD int tables_prepare(const Team& tm, int dim, int n, int rank, const double* F, double* tab,
                         double* N, double* work, int* ipiv, double* sh) {
    const int nn = n * n;
    double* W0 = work;
    double* W1 = work + nn;
    double* W2 = work + 2 * nn;
    double* W3 = work + 3 * nn;
    int status = 0;
    double* L0 = tab;
    double* L1 = tab + nn;
    double* L2 = tab + 2 * nn;
    double* C1 = N;
    double* C2 = N + nn;
    for (int t = tm.tid(); t < 3 * nn; t += tm.size()) tab[t] = 0.0;
    tm.sync();
    if (dim == 2 && rank == 1) {
        // P = A1 (x) B1: T1 = T2 = I/2, Q = I in the same form
        for (int q = 0; q < 2; ++q) {
            for (int t = tm.tid(); t < nn; t += tm.size()) W0[t] = F[q * nn + t];
            tm.sync();
            if (!invert(tm, n, W0, W1, ipiv, sh + 8)) status |= 2;
            for (int t = tm.tid(); t < nn; t += tm.size()) (q ? L1 : L0)[t] = W1[t];
            tm.sync();
        }
        for (int t = tm.tid(); t < nn; t += tm.size()) {
            C1[t] = (t / n == t % n) ? 0.5 : 0.0;
            C2[t] = C1[t];
        }
        tm.sync();
        return status;
    }
    // Pair rotation.  The sum B1 (x) C1 + B2 (x) C2 (3D; A1 (x) B1 + A2 (x) B2 in
    // 2D) is unchanged when (B1, B2) and (C1, C2) are rotated by the same angle
    // after balancing the norms within each term.  The paper inverts the
    // second left and first right factor (Algs. 5 and 7); those can be nearly
    // singular while P is well conditioned, so the angle (one of 8 in [0, pi))
    // that minimises kappa_1 of the two inverted factors is used.
    double* R6 = work + 6 * nn;  // left 1
    double* R7 = work + 7 * nn;  // left 2 (inverted)
    double* R8 = work + 8 * nn;  // right 1 (inverted)
    double* R9 = work + 9 * nn;  // right 2
    {
        const double* l1 = dim == 2 ? F : F + nn;
        const double* l2 = dim == 2 ? F + 2 * nn : F + 3 * nn;
        const double* r1 = dim == 2 ? F + nn : F + 2 * nn;
        const double* r2 = dim == 2 ? F + 3 * nn : F + 4 * nn;
        double p1 = 0.0, p2 = 0.0;
        for (int t = tm.tid(); t < nn; t += tm.size()) {
            p1 += l1[t] * l1[t];
            p2 += l2[t] * l2[t];
        }
        const double s1 = sqrt(tm.sum(p1)), s2 = sqrt(tm.sum(p2));
        const double a1 = s1 > 0.0 ? s1 : 1.0, a2 = s2 > 0.0 ? s2 : 1.0;
        for (int t = tm.tid(); t < nn; t += tm.size()) {
            R6[t] = l1[t] / a1;
            R9[t] = r1[t] * a1;  // temporarily: balanced right 1
            R7[t] = l2[t] / a2;
            R8[t] = r2[t] * a2;  // temporarily: balanced right 2
        }
        tm.sync();
        const double pi = 3.14159265358979323846;
        double best = -1.0;
        int bestk = 0;
        for (int k = 0; k < 8; ++k) {
            const double c = cos(pi * k / 8.0), sn = sin(pi * k / 8.0);
            for (int t = tm.tid(); t < nn; t += tm.size()) {
                W0[t] = -sn * R6[t] + c * R7[t];  // rotated left 2
                W1[t] = c * R9[t] + sn * R8[t];   // rotated right 1
            }
            tm.sync();
            double score = 1.0;
            for (int q = 0; q < 2; ++q) {
                double* M = q == 0 ? W0 : W1;
                const double nm = norm1(tm, n, M, sh);
                const bool ok = invert(tm, n, M, W2, ipiv, sh + 8);
                const double ni = norm1(tm, n, W2, sh);
                score *= ok ? nm * ni : 1e300;
            }
            if (!(score == score)) score = 1e300;
            if (best < 0.0 || score < best) {
                best = score;
                bestk = k;
            }
        }
        const double c = cos(pi * bestk / 8.0), sn = sin(pi * bestk / 8.0);
        for (int t = tm.tid(); t < nn; t += tm.size()) {
            const double bl1 = R6[t], bl2 = R7[t], br1 = R9[t], br2 = R8[t];
            R6[t] = c * bl1 + sn * bl2;
            R7[t] = -sn * bl1 + c * bl2;
            R8[t] = c * br1 + sn * br2;
            R9[t] = -sn * br1 + c * br2;
        }
        tm.sync();
    }
    // factors to invert and to multiply
    const double *Fx, *Fy, *Fz = nullptr, *Gy, *Gz;
    if (dim == 2) {
        Fx = R7;  // A2'
        Fy = R8;  // B1'
        Gy = R6;  // A1'  -> C1 = A2'^{-1} A1'
        Gz = R9;  // B2'  -> C2 = B1'^{-1} B2'
    } else {
        Fx = F;   // A1
        Fy = R7;  // B2'
        Fz = R8;  // C1'
        Gy = R6;  // B1'  -> C1' = B2'^{-1} B1'
        Gz = R9;  // C2'  -> C2' = C1'^{-1} C2'
    }
    // inverses into the L slots: 2D L0 = inv(A2'), L1 = inv(B1');
    // 3D L0 = inv(A1), L1 = inv(B2'), L2 = inv(C1')  (formed in work, then copied)
    double* W4 = work + 4 * nn;
    const double* srcs[3] = {Fx, Fy, Fz};
    double* dsts[3] = {L0, L1, L2};
    for (int q = 0; q < (dim == 3 ? 3 : 2); ++q) {
        for (int t = tm.tid(); t < nn; t += tm.size()) W0[t] = srcs[q][t];
        tm.sync();
        if (!invert(tm, n, W0, W4, ipiv, sh + 8)) status |= 2;
        for (int t = tm.tid(); t < nn; t += tm.size()) dsts[q][t] = W4[t];
        tm.sync();
    }
    // C matrices: 2D: C1 = inv(A2') A1', C2 = inv(B1') B2'.  3D: C1 = inv(B2') B1', C2 = inv(C1') C2'
    const double* invY = dim == 2 ? L0 : L1;
    const double* invZ = dim == 2 ? L1 : L2;
    for (int t = tm.tid(); t < nn; t += tm.size()) {
        W2[t] = invY[t];
        W3[t] = invZ[t];
    }
    tm.sync();
    mm(tm, n, W2, Gy, W0);
    mm(tm, n, W3, Gz, W1);
    for (int t = tm.tid(); t < nn; t += tm.size()) {
        C1[t] = W0[t];
        C2[t] = W1[t];
    }
    tm.sync();
    return status;
}

// finish.  tab holds the inverses (L slots), T1, T2, Q1 = R0, Q2 = R1.
// Work: >= 6 n^2 doubles (T1, T2 and Q's are staged there).
template <class Team>
KP_HD int tables_finish(const Team& tm, int dim, int n, double* tab, double* N, int8_t* kinds,
                        double* work, int* ipiv, double* sh) {
    const int nn = n * n;
    double* W0 = work;
    double* W1 = work + nn;
    double* W4 = work + 2 * nn;
    double* W5 = work + 3 * nn;
    double* T1 = work + 4 * nn;
    double* Qs = work + 5 * nn;
    int status = 0;
    double* Ls[2] = {dim == 2 ? tab : tab + nn, dim == 2 ? tab + nn : tab + 2 * nn};
    const double* Rs[2] = {tab + 3 * nn, tab + 4 * nn};
    const double* T2 = tab + 6 * nn;
    // L = Q^T inverse
    for (int q = 0; q < 2; ++q) {
        for (int t = tm.tid(); t < nn; t += tm.size()) {
            W0[t] = Ls[q][t];
            Qs[t] = Rs[q][t];
        }
        tm.sync();
        mtm(tm, n, Qs, W0, W1);
        for (int t = tm.tid(); t < nn; t += tm.size()) Ls[q][t] = W1[t];
        tm.sync();
    }
    for (int t = tm.tid(); t < nn; t += tm.size()) T1[t] = tab[5 * nn + t];
    // kinds from the standardised T2
    for (int j = tm.tid(); j < n; j += tm.size()) {
        int kd = 0;
        if (j > 0 && T2[j * n + j - 1] != 0.0) kd = 2;
        if (j + 1 < n && T2[(j + 1) * n + j] != 0.0) kd = 1;
        kinds[j] = (int8_t)kd;
    }
    tm.sync();
    // N_j
    for (int j = 0; j < n; ++j) {
        const int kd = kinds[j];
        if (kd == 1) continue;  // filled with its partner
        if (kd == 0) {
            const double tj = T2[j * n + j];
            for (int t = tm.tid(); t < nn; t += tm.size()) W0[t] = T1[t] + ((t / n == t % n) ? tj : 0.0);
            tm.sync();
            if (!invert(tm, n, W0, W1, ipiv, sh + 8)) status |= 2;
            for (int t = tm.tid(); t < nn; t += tm.size()) N[(long)j * nn + t] = W1[t];
            tm.sync();
        } else {
            const double p = T2[j * n + j], q = T2[(j - 1) * n + j], s = T2[j * n + j - 1];
            for (int t = tm.tid(); t < nn; t += tm.size()) W4[t] = T1[t] + ((t / n == t % n) ? p : 0.0);
            tm.sync();
            mm(tm, n, W4, W4, W5);
            for (int t = tm.tid(); t < nn; t += tm.size()) W0[t] = W5[t] - ((t / n == t % n) ? q * s : 0.0);
            tm.sync();
            if (!invert(tm, n, W0, W1, ipiv, sh + 8)) status |= 2;
            for (int t = tm.tid(); t < nn; t += tm.size()) {
                N[(long)j * nn + t] = W1[t];
                N[(long)(j - 1) * nn + t] = W1[t];
            }
            tm.sync();
        }
    }
    // non-finite check (a NaN fails the comparison)
    double bad = 0.0;
    for (long t = tm.tid(); t < 7L * nn; t += tm.size())
        if (!(fabs(tab[t]) < 1e300)) bad = 1.0;
    for (long t = tm.tid(); t < (long)n * nn; t += tm.size())
        if (!(fabs(N[t]) < 1e300)) bad = 1.0;
    if (tm.max(bad) != 0.0) status |= 8;
    return status;
}

// Schur phase for one of the two C matrices: H (n^2 shared, destroyed) holds C;
// T and Q are written to Tout, Qout.
template <class Team>
KP_HD int tables_schur(const Team& tm, int n, const double* C, double* Tout, double* Qout, double* H,
                       double* Q, double* sh) {
    for (int t = tm.tid(); t < n * n; t += tm.size()) H[t] = C[t];
    tm.sync();
    const bool ok = real_schur(tm, n, H, Q, sh);
    for (int t = tm.tid(); t < n * n; t += tm.size()) {
        Tout[t] = H[t];
        Qout[t] = Q[t];
    }
    tm.sync();
    return ok ? 0 : 4;
}

// All three phases in sequence (host checks).  Work: >= 10 n^2 doubles.
template <class Team>
KP_HD int form_tables(const Team& tm, int dim, int n, int rank, const double* F, double* tab,
                      double* N, int8_t* kinds, double* work, int* ipiv, double* sh) {
    const int nn = n * n;
    int status = tables_prepare(tm, dim, n, rank, F, tab, N, work, ipiv, sh);
    status |= tables_schur(tm, n, N, tab + 5 * nn, tab + 3 * nn, work, work + nn, sh);
    status |= tables_schur(tm, n, N + nn, tab + 6 * nn, tab + 4 * nn, work, work + nn, sh);
    status |= tables_finish(tm, dim, n, tab, N, kinds, work, ipiv, sh);
    return status;
}

// ===================================================== generic apply
// z = P^{-1} r for one element and one right-hand side (Alg. 6 / Alg. 8):
// contractions with L0..L(d-1) along each axis, the quasi-triangular Sylvester
// sweep on the last two axes of every slice, contractions with R0, R1 on the
// last two axes.  T is the working precision; Round(v) rounds an operand to
// the storage precision of the tables (identity except for bf16).
struct RoundNone {
    template <typename T>
    KP_HD T operator()(T v) const { return v; }
};
struct RoundBf16 {
    KP_HD float operator()(float v) const { return bf16_to_f32(f32_to_bf16(v)); }
};
// value carried by a split pair hi + lo of bf16 numbers (hi = bf16(v), lo = bf16(v - hi))
struct RoundBf16x2 {
    KP_HD float operator()(float v) const {
        const float hi = bf16_to_f32(f32_to_bf16(v));
        return hi + bf16_to_f32(f32_to_bf16(v - hi));
    }
};

KP_INLINE double ldt(const double* p, long i) { return p[i]; }
KP_INLINE float ldt(const float* p, long i) { return p[i]; }
KP_INLINE float ldt(const uint16_t* p, long i) { return bf16_to_f32(p[i]); }

// out = M (x)_ax X (contraction of axis ax with the n x n matrix M)
template <class Team, typename T, typename TT, class Rnd>
KP_HD void contract_axis(const Team& tm, int dim, int n, int ax, const TT* M, const T* X, T* out,
                         Rnd rnd) {
    int nd = 1;
    for (int i = 0; i < dim; ++i) nd *= n;
    int stride = 1;
    for (int i = ax + 1; i < dim; ++i) stride *= n;
    for (int idx = tm.tid(); idx < nd; idx += tm.size()) {
        const int lo = idx % stride;
        const int i = (idx / stride) % n;
        const int hi = idx / (stride * n);
        const int base = hi * stride * n + lo;
        T acc = (T)0;
#pragma unroll 8
        for (int k = 0; k < n; ++k) acc += (T)ldt(M, i * n + k) * rnd(X[base + k * stride]);
        out[idx] = acc;
    }
    tm.sync();
}


// X: n^d working tensor (holds the result on return); Y, Hs: n^d scratch.
template <class Team, typename T, typename TT, class Rnd>
KP_HD_FORCEINLINE void apply_tensor(const Team& tm, int dim, int n, const TT* tab, const int8_t* kinds, T* X,
                        T* Y, T* Hs, Rnd rnd) {
    const int nn = n * n;
    const TT* L[3] = {tab, tab + nn, tab + 2 * nn};
    const TT* R0 = tab + 3 * nn;
    const TT* R1 = tab + 4 * nn;
    const TT* T1 = tab + 5 * nn;
    const TT* T2 = tab + 6 * nn;
    const TT* N = tab + 7 * nn;
    T* cur = X;
    T* oth = Y;
    // forward contractions
    for (int ax = 0; ax < dim; ++ax) {
        contract_axis(tm, dim, n, ax, L[ax], cur, oth, rnd);
        T* t = cur; cur = oth; oth = t;
    }
    const int ns = dim == 2 ? 1 : n;   // slices
    const int rows = ns * n;           // (slice, i) pairs
    // Sylvester: F = cur (per slice F[i][j] = cur[s*nn + i*n + j]), solution in oth
    T* F = cur;
    T* S = oth;
    int j = n - 1;
    while (j >= 0) {
        const int kd = kinds[j];
        if (kd != 2) {
            const TT* Nj = N + (long)j * nn;
            for (int t = tm.tid(); t < rows; t += tm.size()) {
                const int s = t / n, i = t % n;
                T acc = (T)0;
#pragma unroll 8
                for (int k = 0; k < n; ++k) acc += (T)ldt(Nj, i * n + k) * rnd(F[s * nn + k * n + j]);
                S[s * nn + i * n + j] = acc;
            }
            tm.sync();
            for (int t = tm.tid(); t < rows * j; t += tm.size()) {
                const int k = t % j, si = t / j, s = si / n, i = si % n;
                F[s * nn + i * n + k] -= (T)ldt(T2, k * n + j) * rnd(S[s * nn + i * n + j]);
            }
            tm.sync();
            --j;
        } else {
            const int j1 = j - 1;
            const T p = (T)ldt(T2, j * n + j), q = (T)ldt(T2, j1 * n + j), sv = (T)ldt(T2, j * n + j1);
            const TT* Nj = N + (long)j * nn;
            // Hs[s][0][i] = M g1 - q g2, Hs[s][1][i] = M g2 - s g1, M = T1 + p I
            for (int t = tm.tid(); t < rows; t += tm.size()) {
                const int s = t / n, i = t % n;
                T a1 = (T)0, a2 = (T)0;
#pragma unroll 8
                for (int k = 0; k < n; ++k) {
                    const T tk = (T)ldt(T1, i * n + k);
                    a1 += tk * rnd(F[s * nn + k * n + j1]);
                    a2 += tk * rnd(F[s * nn + k * n + j]);
                }
                const T g1 = F[s * nn + i * n + j1], g2 = F[s * nn + i * n + j];
                Hs[s * 2 * n + i] = a1 + p * g1 - q * g2;
                Hs[s * 2 * n + n + i] = a2 + p * g2 - sv * g1;
            }
            tm.sync();
            for (int t = tm.tid(); t < 2 * rows; t += tm.size()) {
                const int s = t / (2 * n), h = (t / n) % 2, i = t % n;
                T acc = (T)0;
#pragma unroll 8
                for (int k = 0; k < n; ++k) acc += (T)ldt(Nj, i * n + k) * rnd(Hs[s * 2 * n + h * n + k]);
                S[s * nn + i * n + (h ? j : j1)] = acc;
            }
            tm.sync();
            for (int t = tm.tid(); t < rows * j1; t += tm.size()) {
                const int k = t % j1, si = t / j1, s = si / n, i = si % n;
                F[s * nn + i * n + k] -= (T)ldt(T2, k * n + j1) * rnd(S[s * nn + i * n + j1]) +
                                         (T)ldt(T2, k * n + j) * rnd(S[s * nn + i * n + j]);
            }
            tm.sync();
            j -= 2;
        }
    }
    // backward contractions on the last two axes
    contract_axis(tm, dim, n, dim - 2, R0, S, F, rnd);
    contract_axis(tm, dim, n, dim - 1, R1, F, S, rnd);
    if (S != X) {
        const int nd = dim == 2 ? nn : nn * n;
        for (int t = tm.tid(); t < nd; t += tm.size()) X[t] = S[t];
        tm.sync();
    }
}


// ============================================== per-element setup
// Workspace of one element's setup (all shared by the team).
struct SetupWork {
    double* mass;   // n^d
    double* Xax;    // 3 n^2
    double* G;      // n^4 (explicit Gram, when n^2 <= kGramMax)
    double* D1;     // n^4 (3D explicit: stage-1 right factor)
    double* m2;     // n^2 (3D structured: stage-2 block)
    double* X2;     // n^2
    double* Y2;     // n^2
    double* U;      // 3 n^2 Ritz vectors
    double* d;      // n^2 operator scratch
    double* small;  // 64 doubles
    double* Wm;     // (kmax + 16) x n^2 (rank >= 3: R^T of the Lanczos basis and the
                    // block vectors of the refinement; the r unit right vectors at
                    // row kmax + 10)
    double* Vr;     // kmax x kmax (rank >= 3: accumulated Jacobi rotations)
    LanczosWork L;
    const double* Gpre = nullptr;  // explicit blocks: the element's stage-1 Gram, formed beforehand, or null
};
constexpr int kGramMax = 64;  // explicit Gram kept when the left size n^2 <= this

KP_INLINE int lanczos_kmax(int n, bool expl) {
    const int m = n * n;
    int k = expl ? 64 : n + 8;
    return k < m ? k : m;
}

// number of doubles of a SetupWork for (dim, n, explicit, rank)
KP_INLINE long setup_work_doubles(int dim, int n, bool expl, int rank = 2) {
    const long nn = (long)n * n;
    const long m = nn;
    const long kmax = lanczos_kmax(n, expl);
    long t = 0;
    t += (dim == 2 ? nn : nn * n);        // mass
    t += 3 * nn;                          // Xax
    t += (expl && m <= kGramMax) ? m * m : 0;  // G
    t += (expl && dim == 3) ? nn * nn : 0;     // D1
    t += 3 * nn;                          // m2, X2, Y2
    t += 3 * nn;                          // U
    t += nn;                              // d
    t += 64;                              // small
    t += (kmax + 1) * m + m + (kmax + 2) + 2 * (kmax + 1) + 2 * kmax + kmax * kmax + 3 * kmax + 3;
    t += 8;                               // ctrl (as doubles)
    t += 2 * kmax + 4;                    // rot, qc
    if (rank >= 3) t += (kmax + 16) * m + kmax * kmax + kmax + 8;  // Wm (+ block vectors), Vr, norms, order
    return (t + 31) / 32 * 32;
}

KP_INLINE SetupWork carve_setup_work(double* base, int dim, int n, bool expl, int rank = 2) {
    const long nn = (long)n * n;
    const long m = nn;
    const long kmax = lanczos_kmax(n, expl);
    SetupWork W;
    double* p = base;
    W.mass = p; p += (dim == 2 ? nn : nn * n);
    W.Xax = p; p += 3 * nn;
    W.G = p; p += (expl && m <= kGramMax) ? m * m : 0;
    W.D1 = p; p += (expl && dim == 3) ? nn * nn : 0;
    W.m2 = p; p += nn;
    W.X2 = p; p += nn;
    W.Y2 = p; p += nn;
    W.U = p; p += 3 * nn;
    W.d = p; p += nn;
    W.small = p; p += 64;
    W.L.Q = p; p += (kmax + 1) * m;
    W.L.w = p; p += m;
    W.L.qv = nullptr;
    W.L.h = p; p += kmax + 2;
    W.L.alpha = p; p += kmax + 1;
    W.L.beta = p; p += kmax + 1;
    W.L.d = p; p += kmax;
    W.L.e = p; p += kmax;
    W.L.Z = p; p += kmax * kmax;
    W.L.sel = p; p += 3 * kmax;
    W.L.theta = p; p += 3;
    W.L.ctrl = (int*)p; p += 8;
    W.L.rot = p; p += 2 * kmax;
    W.L.qc = (int*)p; p += 4;
    W.Wm = nullptr;
    W.Vr = nullptr;
    if (rank >= 3) {
        W.Wm = p; p += (kmax + 16) * m;
        W.Vr = p; p += kmax * kmax + kmax + 8;
    }
    return W;
}

// Lanczos scalars and the tridiagonal eigenproblem (d, e, Z, sel, h, ...),
// and the operator scratch d, placed in fast shared memory: doubles needed
KP_INLINE long setup_small_doubles(int n, bool expl) {
    const long kmax = lanczos_kmax(n, expl);
    return (kmax + 2) + 2 * (kmax + 1) + 2 * kmax + kmax * kmax + 3 * kmax + 3 + 8 + 2 * kmax + 4 +
           3 * (long)n * n + 64;
}
// the small, often-touched parts of the setup work (in LDS on the GPU): the
// Lanczos scalars and tridiagonal, its work vector and newest basis vector
KP_INLINE void carve_small(double* p, int n, bool expl, SetupWork* W) {
    const long kmax = lanczos_kmax(n, expl);
    W->L.w = p; p += (long)n * n;
    W->L.qv = p; p += (long)n * n;
    W->L.h = p; p += kmax + 2;
    W->L.alpha = p; p += kmax + 1;
    W->L.beta = p; p += kmax + 1;
    W->L.d = p; p += kmax;
    W->L.e = p; p += kmax;
    W->L.Z = p; p += kmax * kmax;
    W->L.sel = p; p += 3 * kmax;
    W->L.theta = p; p += 3;
    W->L.ctrl = (int*)p; p += 8;
    W->L.rot = p; p += 2 * kmax;
    W->L.qc = (int*)p; p += 4;
    W->d = p; p += (long)n * n;
    W->small = p;
}

// start vector of the Lanczos iteration: the caller's guess, else all ones
template <class Team>
KP_HD void lanczos_start(const Team& tm, double* q0, int m, const double* guess) {
    for (int i = tm.tid(); i < m; i += tm.size()) q0[i] = guess ? guess[i] : 1.0;
    tm.sync();
}

// One-sided (Hestenes) Jacobi: rotate pairs of the k columns of Wc (each of
// length len, column c at Wc + c*len) until every pair is orthogonal to
// 1e-15 relative; the rotations are accumulated in Vr (k x k, column c at
// Vr + c*k, set to I here).  The disjoint pairs of one round of a round-robin
// schedule are rotated in parallel, one group (wave) per pair.  Returns false
// if 40 sweeps did not converge.
template <class Team>
KP_HD bool jacobi_orth(const Team& tm, double* Wc, int len, int k, double* Vr) {
    for (int t = tm.tid(); t < k * k; t += tm.size()) Vr[t] = (t / k == t % k) ? 1.0 : 0.0;
    tm.sync();
    if (k < 2) return true;
    const int kk = k + (k & 1);  // even player count; player k is a bye when k is odd
    for (int sweep = 0; sweep < 40; ++sweep) {
        double rotated = 0.0;
        for (int round = 0; round < kk - 1; ++round) {
            for (int pr = tm.group(); pr < kk / 2; pr += tm.groups()) {
                int p, q;
                if (pr == 0) {
                    p = kk - 1;
                    q = round;
                } else {
                    p = (round + pr) % (kk - 1);
                    q = (round - pr + kk - 1) % (kk - 1);
                }
                if (p >= k || q >= k) continue;
                if (p > q) { const int t = p; p = q; q = t; }
                double* wp = Wc + (long)p * len;
                double* wq = Wc + (long)q * len;
                double a = 0.0, b = 0.0, g = 0.0;
                for (int i = tm.lane(); i < len; i += tm.group_size()) {
                    a += wp[i] * wp[i];
                    b += wq[i] * wq[i];
                    g += wp[i] * wq[i];
                }
                a = tm.group_sum(a);
                b = tm.group_sum(b);
                g = tm.group_sum(g);
                if (!(fabs(g) > 1e-15 * sqrt(a * b))) continue;
                const double zeta = (b - a) / (2.0 * g);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
                for (int i = tm.lane(); i < len; i += tm.group_size()) {
                    const double x = wp[i], y = wq[i];
                    wp[i] = c * x - sn * y;
                    wq[i] = sn * x + c * y;
                }
                double* vp = Vr + (long)p * k;
                double* vq = Vr + (long)q * k;
                for (int i = tm.lane(); i < k; i += tm.group_size()) {
                    const double x = vp[i], y = vq[i];
                    vp[i] = c * x - sn * y;
                    vq[i] = sn * x + c * y;
                }
                rotated = 1.0;
            }
            tm.sync();
        }
        if (tm.max(rotated) == 0.0) return true;
    }
    return false;
}

// nrm[c] = ||column c|| for the k columns of Wc; order[0..b) = the b largest (descending)
template <class Team>
KP_HD void column_order(const Team& tm, const double* Wc, int len, int k, int b, double* nrm,
                        int* order) {
    for (int j = tm.group(); j < k; j += tm.groups()) {
        const double* wj = Wc + (long)j * len;
        double a = 0.0;
        for (int i = tm.lane(); i < len; i += tm.group_size()) a += wj[i] * wj[i];
        a = tm.group_sum(a);
        if (tm.lane() == 0) nrm[j] = sqrt(a);
    }
    tm.sync();
    if (tm.leader()) {
        for (int j = 0; j < b; ++j) {
            int best = -1;
            for (int i = 0; i < k; ++i) {
                bool used = false;
                for (int q = 0; q < j; ++q)
                    if (order[q] == i) used = true;
                if (!used && (best < 0 || nrm[i] > nrm[best])) best = i;
            }
            order[j] = best;
        }
    }
    tm.sync();
}

// Accurate top-r singular triplets (rank 3).  The Ritz values of R R^T carry
// absolute errors of order eps sigma_1^2, and the Lanczos vectors that carry
// a small singular direction are formed from products of that size, so a
// third singular value far below the first (down to 1e-6 sigma_1 on these
// blocks) and its vectors lose many digits.  Two steps fix that:
//  1. the Lanczos basis Q_k (built until invariant) is mapped to the right
//     space, Wm = R^T Q_k, and orthogonalised by one-sided Jacobi: the b
//     largest columns give starting triplets;
//  2. two-sided block iteration with b = r + 2 vectors: V = orth(R^T U),
//     U = orth(R V) by one-sided Jacobi, so that R v_i = sigma_i u_i holds as
//     computed; each product with R or R^T has absolute error eps sigma_1
//     only.  Iterates until ||R^T u_i - sigma_i v_i|| <= 32 eps sigma_1 for the
//     r wanted triplets (at most 12 iterations).
// Work: Wm (kmax + 16) x m, Vr kmax^2 + kmax + 8, Q the Lanczos basis (reused).
// Outputs U (r x m) unit left vectors, Vout (r x m) unit right vectors, sig.
template <class Team, class RightOp>
KP_HD bool refine_triplets(const Team& tm, const RightOp& rop, int m, int k, double* Q, int r,
                           double* Wm, double* Vr, double* U, double* Vout, double* sig) {
    double* nrm = Vr + (long)k * k;                 // k
    int* order = (int*)(Vr + (long)k * k + k);      // b ints
    for (int j = 0; j < k; ++j) rop(tm, Q + (long)j * m, 1.0, Wm + (long)j * m);
    bool ok = jacobi_orth(tm, Wm, m, k, Vr);
    const int b = r + 2 < k ? r + 2 : k;
    column_order(tm, Wm, m, k, b, nrm, order);
    // starting left vectors Ub = Q_k p_c into rows [k, k + b) of Wm (Wm rows
    // below k are not read again)
    double* Ub = Wm + (long)k * m;
    for (long t = tm.tid(); t < (long)b * m; t += tm.size()) {
        const int j = (int)(t / m), i = (int)(t % m);
        const int c = order[j];
        double s = 0.0;
        for (int q = 0; q < k; ++q) s += Q[(long)q * m + i] * Vr[(long)c * k + q];
        Ub[t] = s;
    }
    tm.sync();
    // move Ub to the front; Vb, Vn follow (Q is free from here on and serves as Tn)
    double* U0 = Wm;
    double* Vb = Wm + (long)b * m;
    double* Vn = Wm + 2L * b * m;
    double* Tn = Q;
    for (long t = tm.tid(); t < (long)b * m; t += tm.size()) Tn[t] = Ub[t];
    tm.sync();
    for (long t = tm.tid(); t < (long)b * m; t += tm.size()) U0[t] = Tn[t];
    tm.sync();
    double* sg = nrm;   // b singular value estimates (nrm is free again)
    int* ord = order;
    bool conv = false;
    for (int it = 0; it < 12 && !conv; ++it) {
        // Vn = R^T U; residual of the previous pair (R v_i = sg_i u_i holds)
        for (int j = 0; j < b; ++j) rop(tm, U0 + (long)j * m, 1.0, Vn + (long)j * m);
        if (it > 0) {
            double res = 0.0;
            for (int j = tm.group(); j < r; j += tm.groups()) {
                const double* vn = Vn + (long)j * m;
                const double* vb = Vb + (long)j * m;
                double a = 0.0;
                for (int i = tm.lane(); i < m; i += tm.group_size()) {
                    const double d = vn[i] - sg[j] * vb[i];
                    a += d * d;
                }
                a = tm.group_sum(a);
                res = fmax(res, sqrt(a));
            }
            res = tm.max(res);
            if (res <= 32.0 * 2.220446049250313e-16 * sg[0]) conv = true;
        }
        if (conv) break;
        // Vb = orth(Vn) (unit columns)
        ok = jacobi_orth(tm, Vn, m, b, Vr) && ok;
        column_order(tm, Vn, m, b, b, sg, ord);
        for (long t = tm.tid(); t < (long)b * m; t += tm.size()) {
            const int j = (int)(t / m), i = (int)(t % m);
            const int c = ord[j];
            Vb[t] = sg[c] > 0.0 ? Vn[(long)c * m + i] / sg[c] : 0.0;
        }
        tm.sync();
        // Tn = R Vb, orthogonalise; the same rotations keep R (Vb P) = Tn P
        for (int j = 0; j < b; ++j) rop.forward(tm, Vb + (long)j * m, Tn + (long)j * m);
        ok = jacobi_orth(tm, Tn, m, b, Vr) && ok;
        // Vn = Vb P
        for (long t = tm.tid(); t < (long)b * m; t += tm.size()) {
            const int j = (int)(t / m), i = (int)(t % m);
            double s = 0.0;
            for (int q = 0; q < b; ++q) s += Vb[(long)q * m + i] * Vr[(long)j * b + q];
            Vn[t] = s;
        }
        tm.sync();
        column_order(tm, Tn, m, b, b, sg, ord);
        // sorted, normalised: U0 = Tn / sigma, Vb = Vn (both in descending order)
        for (long t = tm.tid(); t < (long)b * m; t += tm.size()) {
            const int j = (int)(t / m), i = (int)(t % m);
            const int c = ord[j];
            U0[t] = sg[c] > 0.0 ? Tn[(long)c * m + i] / sg[c] : 0.0;
            Vb[t] = Vn[(long)c * m + i];
        }
        tm.sync();
        // sg in sorted order (leader), shared
        if (tm.leader()) {
            double tmp[8];
            for (int j = 0; j < b; ++j) tmp[j] = sg[ord[j]];
            for (int j = 0; j < b; ++j) sg[j] = tmp[j];
        }
        tm.sync();
    }
    for (long t = tm.tid(); t < (long)r * m; t += tm.size()) {
        U[t] = U0[t];
        Vout[t] = Vb[t];
    }
    if (tm.leader())
        for (int j = 0; j < r; ++j) sig[j] = sg[j];
    tm.sync();
    return ok && conv;
}

// 2D KSVD of a block given by an operator; writes r factor pairs (A_j, B_j)
// and sigma_j.  Returns status bits.
template <bool kRefine, class Team, class Op, class RightOp>
KP_HD int ksvd_stage(const Team& tm, const Op& op, const RightOp& rop, int n, int r, int kmax,
                     const double* guess, SetupWork& W, double* Aout /* r n^2, stride sa */,
                     long sa, double* Bout, long sb, int sdim_right, double* sigma) {
    const int m = n * n;
    lanczos_start(tm, W.L.Q, m, guess);
    if (kRefine && r >= 3 && W.Wm) {
        const int ok = lanczos_top(tm, op, m, r, kmax, 1e-14, W.L, W.U, true);
        const int k = W.L.ctrl[1];
        double* sg = W.small;
        double* V = W.Wm + (long)(kmax + 10) * m;
        const bool jc = refine_triplets(tm, rop, m, k, W.L.Q, r, W.Wm, W.Vr, W.U, V, sg);
        for (int j = 0; j < r; ++j) {
            double* u = W.U + (long)j * m;
            const double* v = V + (long)j * m;
            const double sgn = canonical_sign(tm, u, m, W.L.ctrl + 2);
            const double rs = sqrt(sg[j]);
            if (tm.leader()) sigma[j] = sg[j];
            for (int i = tm.tid(); i < m; i += tm.size()) {
                Aout[j * sa + i] = rs * u[i];
                Bout[j * sb + i] = sgn * rs * v[i];
            }
            tm.sync();
        }
        (void)sdim_right;
        return (ok && jc) ? 0 : 1;
    }
    const int conv = lanczos_top(tm, op, m, r, kmax, 1e-14, W.L, W.U);
    int status = conv ? 0 : 1;
    for (int j = 0; j < r; ++j) {
        double* u = W.U + (long)j * m;
        canonical_sign(tm, u, m, W.L.ctrl + 2);
        // sigma_j = ||R^T u_j|| rather than sqrt(theta_j): the Gram eigenvalue
        // carries an absolute error of order eps * sigma_1^2, which would cost
        // sigma_j relative accuracy (sigma_1 / sigma_j)^2 eps; the norm of the
        // right vector loses only a factor sigma_1 / sigma_j.
        double* B = Bout + j * sb;
        rop(tm, u, 1.0, B);
        const int mr = sdim_right * sdim_right;  // right factor entries (m when both sides are n x n)
        double p = 0.0;
        for (int i = tm.tid(); i < mr; i += tm.size()) p += B[i] * B[i];
        const double sg = sqrt(tm.sum(p));
        const double rs = sqrt(sg);
        const double inv = rs > 0.0 ? 1.0 / rs : 0.0;
        if (tm.leader()) sigma[j] = sg;
        for (int i = tm.tid(); i < m; i += tm.size()) Aout[j * sa + i] = rs * u[i];
        for (int i = tm.tid(); i < mr; i += tm.size()) B[i] *= inv;
        tm.sync();
    }
    tm.sync();
    return status;
}

// R^T (operator()) and R (forward) of one block on left / right vectors
struct RightStruct2 {
    const OpStruct2* op;
    template <class Team>
    KP_HD void operator()(const Team& tm, const double* x, double sc, double* B) const {
        op->right_factor(tm, x, sc, B);
    }
    template <class Team>
    KP_HD void forward(const Team& tm, const double* v, double* y) const {
        op->forward(tm, v, y);
    }
};
struct RightStream {
    const OpStream* op;
    template <class Team>
    KP_HD void operator()(const Team& tm, const double* x, double sc, double* B) const {
        op->right_factor(tm, x, sc, B);
    }
    template <class Team>
    KP_HD void forward(const Team& tm, const double* v, double* y) const {
        op->forward(tm, v, y);
    }
};

KP_INLINE double struct2_normY2(int n, const double* Y) {
    double s = 0.0;
    for (int t = 0; t < n * n; ++t) s += Y[t] * Y[t];
    return s;
}
KP_INLINE double struct3_nrm2(int n, const double* Y, const double* Z, const double* w) {
    double y2 = 0.0, z2 = 0.0, w2 = 0.0, ty = 0.0, tz = 0.0;
    for (int t = 0; t < n * n; ++t) { y2 += Y[t] * Y[t]; z2 += Z[t] * Z[t]; }
    for (int i = 0; i < n; ++i) {
        w2 += w[i] * w[i];
        ty += Y[i * n + i] * w[i];
        tz += Z[i * n + i] * w[i];
    }
    return y2 * w2 + w2 * z2 + 2.0 * ty * tz;
}

// Full setup of one element (Alg. 5 / Alg. 7, first steps): factors
// ([A1,B1,A2,B2,..] in 2D, [A1,B1,C1,B2,C2] in 3D) and singular values.
// block: the explicit block, or null for the structured (matrix-free) form
// of rec.  guess: Lanczos start (left vector of the first stage) or null;
// guess2: 3D only, Lanczos start of the second stage (vec B1) or null.
// kRefine: compile the rank >= 3 refinement (2D) into this instance
template <bool kRefine, class Team>
KP_HD int setup_element(const Team& tm, int dim, int n, int rank, const Tables1D& T,
                        const double* rec, const double* block, const double* guess,
                        double* factors, double* sigma, SetupWork& W,
                        const double* guess2 = nullptr) {
    const int nn = n * n;
    const bool expl = block != nullptr;
    const int kmax = lanczos_kmax(n, expl);
    int status = 0;
    if (!expl) record_structure(tm, rec, T, dim, W.mass, W.Xax);
    for (int j = tm.tid(); j < 4; j += tm.size()) sigma[j] = 0.0;
    tm.sync();
    if (dim == 2) {
        if (expl) {
            OpStream st{n, n, block, W.d};
            RightStream rs{&st};
            if (nn <= kGramMax) {
                const double* G1 = W.Gpre;
                if (!G1) {
                    explicit_gram(tm, n, n, block, W.G);
                    G1 = W.G;
                }
                OpGram og{nn, G1};
                status |= ksvd_stage<kRefine>(tm, og, rs, n, rank, kmax, guess, W, factors, 2L * nn,
                                     factors + nn, 2L * nn, n, sigma);
            } else {
                status |= ksvd_stage<kRefine>(tm, st, rs, n, rank, kmax, guess, W, factors, 2L * nn,
                                     factors + nn, 2L * nn, n, sigma);
            }
        } else {
            OpStruct2 op{n, W.mass, W.Xax, W.Xax + nn, T.w, W.d, nullptr,
                         struct2_normY2(n, W.Xax + nn)};
            RightStruct2 rs{&op};
            status |= ksvd_stage<kRefine>(tm, op, rs, n, rank, kmax, guess, W, factors, 2L * nn,
                                 factors + nn, 2L * nn, n, sigma);
        }
        return status;
    }
    // ---- 3D, stage 1: A ~ A1 (x) D1
    double sig1[4];
    if (expl) {
        if (nn > kGramMax) return 64;  // unsupported size for explicit 3D
        const double* G1 = W.Gpre;
        if (!G1) {
            explicit_gram(tm, n, nn, block, W.G);
            G1 = W.G;
        }
        OpGram og{nn, G1};
        lanczos_start(tm, W.L.Q, nn, guess);
        const int conv = lanczos_top(tm, og, nn, 1, kmax, 1e-14, W.L, W.U);
        status |= conv ? 0 : 1;
    } else {
        OpStruct3 op{n, W.mass, W.Xax, W.Xax + nn, W.Xax + 2 * nn, T.w, W.d,
                     struct3_nrm2(n, W.Xax + nn, W.Xax + 2 * nn, T.w)};
        op.precompute(tm, W.d, W.small);  // the mass tensor is then read once
        lanczos_start(tm, W.L.Q, nn, guess);
        const int conv = lanczos_top(tm, op, nn, 1, kmax, 1e-14, W.L, W.U);
        status |= conv ? 0 : 1;
    }
    canonical_sign(tm, W.U, nn, W.L.ctrl + 2);
    const double th = W.L.theta[0];
    sig1[0] = sqrt(th > 0.0 ? th : 0.0);
    const double rs1 = sqrt(sig1[0]);
    if (tm.leader()) sigma[0] = sig1[0];
    for (int i = tm.tid(); i < nn; i += tm.size()) factors[i] = rs1 * W.U[i];  // A1
    tm.sync();
    const double sc = rs1 > 0.0 ? 1.0 / rs1 : 0.0;
    // ---- stage 2: D1 ~ B1 (x) C1 + B2 (x) C2 ; factors B1 at 1, C1 at 2, B2 at 3, C2 at 4
    const int kmax2 = lanczos_kmax(n, expl);
    if (expl) {
        OpStream st1{n, nn, block, W.d};
        st1.right_factor(tm, W.U, sc, W.D1);
        OpStream st2{n, n, W.D1, W.d};
        RightStream rs2{&st2};
        explicit_gram(tm, n, n, W.D1, W.G);
        OpGram og{nn, W.G};
        status |= ksvd_stage<false>(tm, og, rs2, n, 2, kmax2, guess2, W, factors + nn, 2L * nn,
                             factors + 2 * nn, 2L * nn, n, sigma + 1);
    } else {
        OpStruct3 op{n, W.mass, W.Xax, W.Xax + nn, W.Xax + 2 * nn, T.w, W.d, 0.0};
        op.right_factor(tm, W.U, sc, W.m2, W.X2, W.Y2);
        OpStruct2 op2{n, W.m2, W.X2, W.Y2, T.w, W.d, nullptr, struct2_normY2(n, W.Y2)};
        RightStruct2 rs2{&op2};
        status |= ksvd_stage<false>(tm, op2, rs2, n, 2, kmax2, guess2, W, factors + nn, 2L * nn,
                             factors + 2 * nn, 2L * nn, n, sigma + 1);
    }
    return status;
}

}  // namespace kp
