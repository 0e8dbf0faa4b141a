// Acceptance test of predicted Kronecker factors (learned setup).
//
// For the structured block of an element record (elem_ops.h,
// record_structure) and a predicted factor stack F (3D: A1,B1,C1,B2,C2; 2D:
// A1,B1,A2,B2), computes
//   res   = ||A - P(F)||_F^2 = ||A||^2 - 2 <A, P> + ||P||^2, all in closed form
//           from the structure (no block is formed);
//   proxy = ||A||^2 - (energy of the best completion of F's left subspaces):
//           2D: U = orth[vec A1, vec A2], energy = ||R(A)^T U||_F^2;
//           3D: u = vec A1 / ||A1||, D = unvec(R(A)^T u) (a structured 2D
//           block), U2 = orth[vec B1, vec B2], energy = ||R(D)^T U2||_F^2.
// The proxy completes the predicted subspaces optimally, so it never exceeds
// the optimum's residual by more than the subspaces' error, and it equals the
// SVD residual on the SVD's own subspaces.  The prediction is accepted when
// res <= factor * proxy + 1e-12 ||A||^2 and res < ||A||^2.
#pragma once

#include "elem_ops.h"

namespace kp {

// element status bits of the learned path (the values of KP_ELEM_LEARNED_*)
constexpr int kStatusLearnedRejected = 16;
constexpr int kStatusLearnedWarm = 32;

// sum_i w_i M_ii and <M, N> for n x n row-major matrices (team reductions)
template <class Team>
KP_HD double wdiag(const Team& tm, int n, const double* w, const double* M) {
    double p = 0.0;
    for (int i = tm.tid(); i < n; i += tm.size()) p += w[i] * M[i * n + i];
    return tm.sum(p);
}
template <class Team>
KP_HD double frob_dot(const Team& tm, int nn, const double* M, const double* N) {
    double p = 0.0;
    for (int t = tm.tid(); t < nn; t += tm.size()) p += M[t] * N[t];
    return tm.sum(p);
}

// ||A||^2 of the structured block: diagonal entries plus the off-diagonal
// entries of each axis operator (each appears once per combination of the
// other axes' diagonal W entries).
template <class Team>
KP_HD double struct_norm2(const Team& tm, int dim, int n, const double* m, const double* Xax,
                          const double* w) {
    const int nn = n * n;
    const long nd = dim == 2 ? nn : (long)nn * n;
    double p = 0.0;
    for (long t = tm.tid(); t < nd; t += tm.size()) {
        double v = m[t];
        if (dim == 2) {
            const int i = (int)(t / n), k = (int)(t % n);
            v += Xax[i * n + i] * w[k] + w[i] * Xax[nn + k * n + k];
        } else {
            const int i = (int)(t / nn), j = (int)((t / n) % n), k = (int)(t % n);
            v += Xax[i * n + i] * w[j] * w[k] + w[i] * Xax[nn + j * n + j] * w[k] +
                 w[i] * w[j] * Xax[2 * nn + k * n + k];
        }
        p += v * v;
    }
    double off = 0.0;
    for (int t = tm.tid(); t < dim * nn; t += tm.size()) {
        const int q = t % nn;
        if (q / n != q % n) off += Xax[t] * Xax[t];
    }
    double w2 = 0.0;
    for (int i = 0; i < n; ++i) w2 += w[i] * w[i];
    const double wp = dim == 2 ? w2 : w2 * w2;
    return tm.sum(p) + wp * tm.sum(off);
}

// <A, M1 (x) M2 [(x) M3]> of the structured block
template <class Team>
KP_HD double struct_inner(const Team& tm, int dim, int n, const double* m, const double* Xax,
                          const double* w, const double* M1, const double* M2, const double* M3) {
    const int nn = n * n;
    double p = 0.0;
    if (dim == 2) {
        for (int t = tm.tid(); t < nn; t += tm.size()) {
            const int i = t / n, k = t % n;
            p += m[t] * M1[i * n + i] * M2[k * n + k];
        }
        const double dm = tm.sum(p);
        return dm + frob_dot(tm, nn, Xax, M1) * wdiag(tm, n, w, M2) +
               wdiag(tm, n, w, M1) * frob_dot(tm, nn, Xax + nn, M2);
    }
    for (int t = tm.tid(); t < nn * n; t += tm.size()) {
        const int i = t / nn, j = (t / n) % n, k = t % n;
        p += m[t] * M1[i * n + i] * M2[j * n + j] * M3[k * n + k];
    }
    const double dm = tm.sum(p);
    const double w1 = wdiag(tm, n, w, M1), w2 = wdiag(tm, n, w, M2), w3 = wdiag(tm, n, w, M3);
    return dm + frob_dot(tm, nn, Xax, M1) * w2 * w3 + w1 * frob_dot(tm, nn, Xax + nn, M2) * w3 +
           w1 * w2 * frob_dot(tm, nn, Xax + 2 * nn, M3);
}

// orthonormalise two vectors of length len in place (Gram-Schmidt twice);
// a zero vector stays zero
template <class Team>
KP_HD void orth2(const Team& tm, int len, double* a, double* b) {
    double na = sqrt(frob_dot(tm, len, a, a));
    const double ia = na > 0.0 ? 1.0 / na : 0.0;
    for (int t = tm.tid(); t < len; t += tm.size()) a[t] *= ia;
    tm.sync();
    for (int pass = 0; pass < 2; ++pass) {
        const double h = frob_dot(tm, len, a, b);
        for (int t = tm.tid(); t < len; t += tm.size()) b[t] -= h * a[t];
        tm.sync();
    }
    const double nb = sqrt(frob_dot(tm, len, b, b));
    const double ib = nb > 0.0 ? 1.0 / nb : 0.0;
    for (int t = tm.tid(); t < len; t += tm.size()) b[t] *= ib;
    tm.sync();
}

// Work: mass n^d, Xax 3 n^2, then 8 n^2 + n doubles.  out[0] = res,
// out[1] = proxy, out[2] = ||A||^2, out[3..5] = Rayleigh-Ritz singular value
// estimates (3D: ||D||, then the two stage-2 values; 2D: the two values).
template <class Team>
KP_HD bool learned_check(const Team& tm, int dim, int n, const Tables1D& T, const double* rec,
                         const double* F, double* mass, double* Xax, double* work, double factor,
                         double* out) {
    const int nn = n * n;
    record_structure(tm, rec, T, dim, mass, Xax);
    const double a2 = struct_norm2(tm, dim, n, mass, Xax, T.w);
    double res, energy;
    double* q1 = work;
    double* q2 = work + nn;
    double* Wt = work + 2 * nn;
    double* m2 = work + 3 * nn;
    double* X2 = work + 4 * nn;
    double* Y2 = work + 5 * nn;
    double* dsc = work + 6 * nn;   // n^2 operator scratch
    double s1, s2, s0 = 0.0;
    if (dim == 2) {
        const double *A1 = F, *B1 = F + nn, *A2 = F + 2 * nn, *B2 = F + 3 * nn;
        const double ip = struct_inner(tm, 2, n, mass, Xax, T.w, A1, B1, nullptr) +
                          struct_inner(tm, 2, n, mass, Xax, T.w, A2, B2, nullptr);
        const double p2 = frob_dot(tm, nn, A1, A1) * frob_dot(tm, nn, B1, B1) +
                          frob_dot(tm, nn, A2, A2) * frob_dot(tm, nn, B2, B2) +
                          2.0 * frob_dot(tm, nn, A1, A2) * frob_dot(tm, nn, B1, B2);
        res = a2 - 2.0 * ip + p2;
        for (int t = tm.tid(); t < nn; t += tm.size()) {
            q1[t] = A1[t];
            q2[t] = A2[t];
        }
        tm.sync();
        orth2(tm, nn, q1, q2);
        OpStruct2 op{n, mass, Xax, Xax + nn, T.w, dsc, nullptr, struct2_normY2(n, Xax + nn)};
        op.right_factor(tm, q1, 1.0, Wt);
        s1 = sqrt(frob_dot(tm, nn, Wt, Wt));
        op.right_factor(tm, q2, 1.0, Wt);
        s2 = sqrt(frob_dot(tm, nn, Wt, Wt));
    } else {
        const double *A1 = F, *B1 = F + nn, *C1 = F + 2 * nn, *B2 = F + 3 * nn, *C2 = F + 4 * nn;
        const double ip = struct_inner(tm, 3, n, mass, Xax, T.w, A1, B1, C1) +
                          struct_inner(tm, 3, n, mass, Xax, T.w, A1, B2, C2);
        const double p2 = frob_dot(tm, nn, A1, A1) *
                          (frob_dot(tm, nn, B1, B1) * frob_dot(tm, nn, C1, C1) +
                           frob_dot(tm, nn, B2, B2) * frob_dot(tm, nn, C2, C2) +
                           2.0 * frob_dot(tm, nn, B1, B2) * frob_dot(tm, nn, C1, C2));
        res = a2 - 2.0 * ip + p2;
        // stage 1: D = R(A)^T u, u = vec A1 / ||A1||, as the structured 2D block (m2, X2, Y2)
        const double na = sqrt(frob_dot(tm, nn, A1, A1));
        const double ia = na > 0.0 ? 1.0 / na : 0.0;
        for (int t = tm.tid(); t < nn; t += tm.size()) q1[t] = A1[t] * ia;
        tm.sync();
        OpStruct3 op{n, mass, Xax, Xax + nn, Xax + 2 * nn, T.w, dsc, 0.0};
        op.right_factor(tm, q1, 1.0, m2, X2, Y2);
        s0 = sqrt(struct_norm2(tm, 2, n, m2, X2, T.w));
        // stage 2 on D with U2 = orth[vec B1, vec B2]
        for (int t = tm.tid(); t < nn; t += tm.size()) {
            q1[t] = B1[t];
            q2[t] = B2[t];
        }
        tm.sync();
        orth2(tm, nn, q1, q2);
        OpStruct2 op2{n, m2, X2, Y2, T.w, dsc, nullptr, struct2_normY2(n, Y2)};
        op2.right_factor(tm, q1, 1.0, Wt);
        s1 = sqrt(frob_dot(tm, nn, Wt, Wt));
        op2.right_factor(tm, q2, 1.0, Wt);
        s2 = sqrt(frob_dot(tm, nn, Wt, Wt));
    }
    energy = s1 * s1 + s2 * s2;
    const double proxy = a2 - energy;
    if (tm.leader()) {
        out[0] = res;
        out[1] = proxy;
        out[2] = a2;
        out[3] = dim == 3 ? s0 : s1;
        out[4] = dim == 3 ? s1 : s2;
        out[5] = dim == 3 ? s2 : 0.0;
    }
    tm.sync();
    // a prediction that explains nothing (res >= ||A||^2, e.g. all zeros, where
    // the proxy degenerates to ||A||^2 as well) is never accepted
    return res <= factor * proxy + 1e-12 * a2 && res < a2;
}

}  // namespace kp
