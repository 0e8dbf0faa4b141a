// Acceptance test of predicted Kronecker factors (learned setup).
//
// The SVD's factors judge a prediction.  For the structured block A of an
// element record (elem_ops.h, record_structure), a predicted factor stack Fp
// and the SVD's stack Fs (3D: A1,B1,C1,B2,C2; 2D: A1,B1,A2,B2) with the SVD
// preconditioner's FP64 apply tables:
//   res_p = ||A - P(Fp)||_F and res_s = ||A - P(Fs)||_F, in closed form from
//           the structure (||A||^2 - 2 <A, P> + ||P||^2; no block is formed);
//   gamma = a power estimate of ||P(Fs)^{-1} P(Fp) - I||_2: from the
//           normalised ones vector v_0, e_k = P(Fs)^{-1} P(Fp) v_k - v_k,
//           gamma = max_k ||e_k||, v_{k+1} = e_k / ||e_k|| (steps k < 3);
//           every ||e_k|| is a lower bound of the norm.
// The prediction is used when res_p <= factor * res_s (the rearranged
// residual within factor times the SVD's, Sec. 4.1), res_p < ||A||_F (it
// explains part of A), and gamma <= guard.  A Frobenius residual says nothing
// about an eigenvalue sum of the Kronecker sum near zero; with
// ||P(Fs)^{-1} P(Fp) - I|| <= g < 1 the preconditioned operators of the two
// factor sets differ by at most g / (1 - g) relatively.
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

// ||A - P(F)||_F^2 of the structured block (closed form); a2 = ||A||_F^2
template <class Team>
KP_HD double struct_residual2(const Team& tm, int dim, int n, const double* m, const double* Xax,
                              const double* w, const double* F, double a2) {
    const int nn = n * n;
    if (dim == 2) {
        const double *A1 = F, *B1 = F + nn, *A2 = F + 2 * nn, *B2 = F + 3 * nn;
        const double ip = struct_inner(tm, 2, n, m, Xax, w, A1, B1, nullptr) +
                          struct_inner(tm, 2, n, m, Xax, w, A2, B2, nullptr);
        const double p2 = frob_dot(tm, nn, A1, A1) * frob_dot(tm, nn, B1, B1) +
                          frob_dot(tm, nn, A2, A2) * frob_dot(tm, nn, B2, B2) +
                          2.0 * frob_dot(tm, nn, A1, A2) * frob_dot(tm, nn, B1, B2);
        return a2 - 2.0 * ip + p2;
    }
    const double *A1 = F, *B1 = F + nn, *C1 = F + 2 * nn, *B2 = F + 3 * nn, *C2 = F + 4 * nn;
    const double ip = struct_inner(tm, 3, n, m, Xax, w, A1, B1, C1) + struct_inner(tm, 3, n, m, Xax, w, A1, B2, C2);
    const double p2 = frob_dot(tm, nn, A1, A1) *
                      (frob_dot(tm, nn, B1, B1) * frob_dot(tm, nn, C1, C1) +
                       frob_dot(tm, nn, B2, B2) * frob_dot(tm, nn, C2, C2) +
                       2.0 * frob_dot(tm, nn, B1, B2) * frob_dot(tm, nn, C1, C2));
    return a2 - 2.0 * ip + p2;
}

// W = P(F) V for the rank-2 stack F (2D: A1(x)B1 + A2(x)B2; 3D:
// A1(x)(B1(x)C1 + B2(x)C2)); X, Y: n^d scratch
template <class Team>
KP_HD void kron_apply(const Team& tm, int dim, int n, const double* F, const double* V, double* W, double* X,
                      double* Y) {
    const int nn = n * n;
    const long nd = dim == 2 ? nn : (long)nn * n;
    RoundNone rn;
    if (dim == 2) {
        contract_axis(tm, 2, n, 1, F + nn, V, X, rn);
        contract_axis(tm, 2, n, 0, F, X, W, rn);
        contract_axis(tm, 2, n, 1, F + 3 * nn, V, X, rn);
        contract_axis(tm, 2, n, 0, F + 2 * nn, X, Y, rn);
        for (long t = tm.tid(); t < nd; t += tm.size()) W[t] += Y[t];
        tm.sync();
        return;
    }
    contract_axis(tm, 3, n, 2, F + 2 * nn, V, X, rn);
    contract_axis(tm, 3, n, 1, F + nn, X, Y, rn);
    contract_axis(tm, 3, n, 2, F + 4 * nn, V, X, rn);
    contract_axis(tm, 3, n, 1, F + 3 * nn, X, W, rn);
    for (long t = tm.tid(); t < nd; t += tm.size()) W[t] += Y[t];
    tm.sync();
    contract_axis(tm, 3, n, 0, F, W, X, rn);
    for (long t = tm.tid(); t < nd; t += tm.size()) W[t] = X[t];
    tm.sync();
}

constexpr int kGuardSteps = 3;

// number of doubles of the judge's scratch: X, Y, V, W (n^d each), Hs (2 n^2),
// Xax (3 n^2)
KP_INLINE long judge_work_doubles(int dim, int n) {
    const long nn = (long)n * n;
    const long nd = dim == 2 ? nn : nn * n;
    return 4 * nd + 5 * nn;
}

// out[0..4) = res_p, res_s, ||A||_F, gamma (Frobenius norms, not squares).
// tab / kinds: the element's FP64 apply tables of the SVD factors Fs.
template <class Team>
KP_HD bool learned_judge(const Team& tm, int dim, int n, const Tables1D& T, const double* rec, const double* Fp,
                         const double* Fs, const double* tab, const int8_t* kinds, double* work, double factor,
                         double guard, double* out) {
    const int nn = n * n;
    const long nd = dim == 2 ? nn : (long)nn * n;
    double* X = work;
    double* Y = X + nd;
    double* V = Y + nd;
    double* W = V + nd;
    double* Hs = W + nd;
    double* Xax = Hs + 2 * nn;
    record_structure(tm, rec, T, dim, X, Xax);
    const double a2 = struct_norm2(tm, dim, n, X, Xax, T.w);
    const double rp2 = struct_residual2(tm, dim, n, X, Xax, T.w, Fp, a2);
    const double rs2 = struct_residual2(tm, dim, n, X, Xax, T.w, Fs, a2);
    const double rp = sqrt(rp2 > 0.0 ? rp2 : 0.0), rs = sqrt(rs2 > 0.0 ? rs2 : 0.0), a = sqrt(a2);
    tm.sync();
    const double v0 = 1.0 / sqrt((double)nd);
    for (long t = tm.tid(); t < nd; t += tm.size()) V[t] = v0;
    tm.sync();
    double gamma = 0.0;
    for (int k = 0; k < kGuardSteps; ++k) {
        kron_apply(tm, dim, n, Fp, V, W, X, Y);
        for (long t = tm.tid(); t < nd; t += tm.size()) X[t] = W[t];
        tm.sync();
        apply_tensor(tm, dim, n, tab, kinds, X, Y, Hs, RoundNone());
        double p = 0.0;
        for (long t = tm.tid(); t < nd; t += tm.size()) {
            const double e = X[t] - V[t];
            X[t] = e;
            p += e * e;
        }
        const double ne = sqrt(tm.sum(p));
        if (!(ne == ne)) {   // NaN: the prediction is not finite
            gamma = ne;
            break;
        }
        gamma = ne > gamma ? ne : gamma;
        if (!(ne > 0.0)) break;
        const double inv = 1.0 / ne;
        for (long t = tm.tid(); t < nd; t += tm.size()) V[t] = X[t] * inv;
        tm.sync();
    }
    if (tm.leader()) {
        out[0] = rp;
        out[1] = rs;
        out[2] = a;
        out[3] = gamma;
    }
    tm.sync();
    return rp <= factor * rs && rp < a && gamma <= guard;
}

}  // namespace kp
