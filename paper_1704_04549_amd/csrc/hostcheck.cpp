// Host build of the per-element routines of elem_ops.h with a one-thread team.
//
// This library exists only so the CPU test suite can check the arithmetic the
// GPU kernels run (same source, same operation order within each thread)
// without a GPU.  The product library (libkp.so) neither links nor loads it.
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "elem_ops.h"
#include "rank3.h"
#include "learned.h"
#include "quad.h"
#include "sys.h"
#include "tables.h"

using namespace kp;

extern "C" {

int kph_make_tables(int n, double* x, double* w, double* D, double* S, double* K, double* l0,
                    double* l1) {
    Tables1D t;
    if (!make_tables(n, &t)) return 1;
    memcpy(x, t.x, n * sizeof(double));
    memcpy(w, t.w, n * sizeof(double));
    memcpy(l0, t.l0, n * sizeof(double));
    memcpy(l1, t.l1, n * sizeof(double));
    memcpy(D, t.D, n * n * sizeof(double));
    memcpy(S, t.S, n * n * sizeof(double));
    memcpy(K, t.K, n * n * sizeof(double));
    return 0;
}

int kph_block(int dim, int n, const double* rec, double* out) {
    Tables1D t;
    if (!make_tables(n, &t)) return 1;
    HostTeam tm;
    const long nd = dim == 2 ? n * n : n * n * n;
    std::vector<double> mass(nd), Xax(3 * n * n);
    record_structure(tm, rec, t, dim, mass.data(), Xax.data());
    for (long I = 0; I < nd; ++I)
        for (long J = 0; J < nd; ++J) out[I * nd + J] = block_entry(dim, n, I, J, mass.data(), Xax.data(), t.w);
    return 0;
}

int kph_setup(int dim, int n, int rank, const double* rec, const double* block, const double* guess,
              double* factors, double* sigma, int* steps) {
    Tables1D t;
    if (!make_tables(n, &t)) return -1;
    HostTeam tm;
    const bool expl = block != nullptr;
    std::vector<double> ws(setup_work_doubles(dim, n, expl, rank) + 64, 0.0);
    SetupWork W = carve_setup_work(ws.data(), dim, n, expl, rank);
    int st = rank >= 3 ? setup_element<true>(tm, dim, n, rank, t, rec, block, guess, factors, sigma, W)
                       : setup_element<false>(tm, dim, n, rank, t, rec, block, guess, factors, sigma, W);
    if (steps) *steps = W.L.ctrl[1];
    return st;
}

int kph_form_tables(int dim, int n, int rank, const double* factors, double* tab, int8_t* kinds) {
    HostTeam tm;
    std::vector<double> work(10 * n * n + 64);
    std::vector<int> piv(n + 1);
    double sh[kMaxN + 8];
    return form_tables(tm, dim, n, rank, factors, tab, tab + 7L * n * n, kinds, work.data(), piv.data(), sh);
}

// prec 0: FP64; 1: FP32; 2: BF16 operands with FP32 accumulation; 3: split BF16 (hi + lo)
int kph_apply(int dim, int n, int prec, const double* tab, const int8_t* kinds, const double* r,
              double* z) {
    HostTeam tm;
    const long nd = dim == 2 ? n * n : n * n * n;
    const long ne = tab_entries(n);
    if (prec == 0) {
        std::vector<double> X(r, r + nd), Y(nd), H(2 * nd);
        apply_tensor(tm, dim, n, tab, kinds, X.data(), Y.data(), H.data(), RoundNone());
        memcpy(z, X.data(), nd * sizeof(double));
    } else if (prec == 1) {
        std::vector<float> tf(ne), X(nd), Y(nd), H(2 * nd);
        for (long i = 0; i < ne; ++i) tf[i] = (float)tab[i];
        for (long i = 0; i < nd; ++i) X[i] = (float)r[i];
        apply_tensor(tm, dim, n, tf.data(), kinds, X.data(), Y.data(), H.data(), RoundNone());
        for (long i = 0; i < nd; ++i) z[i] = X[i];
    } else if (prec == 3) {
        std::vector<float> tf(ne), X(nd), Y(nd), H(2 * nd);
        RoundBf16x2 rx;
        for (long i = 0; i < ne; ++i) tf[i] = rx((float)tab[i]);
        for (long i = 0; i < nd; ++i) X[i] = (float)r[i];
        apply_tensor(tm, dim, n, tf.data(), kinds, X.data(), Y.data(), H.data(), rx);
        for (long i = 0; i < nd; ++i) z[i] = X[i];
    } else {
        std::vector<uint16_t> tb(ne);
        std::vector<float> X(nd), Y(nd), H(2 * nd);
        for (long i = 0; i < ne; ++i) tb[i] = f32_to_bf16((float)tab[i]);
        for (long i = 0; i < nd; ++i) X[i] = (float)r[i];
        apply_tensor(tm, dim, n, tb.data(), kinds, X.data(), Y.data(), H.data(), RoundBf16());
        for (long i = 0; i < nd; ++i) z[i] = X[i];
    }
    return 0;
}

// rank-3 2D apply: F = A1,B1,A2,B2,A3,B3; tab / kinds = rank-2 tables.
// Returns the inner iteration count (negative if the target was missed).
int kph_apply_rank3(int n, int prec, const double* F, const double* tab, const int8_t* kinds,
                    const double* r, double* z, int m) {
    HostTeam tm;
    const long nn = (long)n * n;
    const long ne = tab_entries(n);
    std::vector<double> work(rank3_work_doubles(n, m)), small(rank3_small_doubles(m));
    const double rtol = rank3_rtol(prec);
    if (prec == 0) {
        std::vector<double> tw(3 * nn);
        return rank3_solve(tm, n, F, tab, kinds, r, z, work.data(), tw.data(), small.data(), m, rtol,
                           kRank3MaxIters, RoundNone());
    }
    std::vector<float> tw(3 * nn);
    if (prec == 1) {
        std::vector<float> tf(ne);
        for (long i = 0; i < ne; ++i) tf[i] = (float)tab[i];
        return rank3_solve(tm, n, F, tf.data(), kinds, r, z, work.data(), tw.data(), small.data(), m,
                           rtol, kRank3MaxIters, RoundNone());
    }
    if (prec == 3) {
        std::vector<float> tf(ne);
        RoundBf16x2 rx;
        for (long i = 0; i < ne; ++i) tf[i] = rx((float)tab[i]);
        return rank3_solve(tm, n, F, tf.data(), kinds, r, z, work.data(), tw.data(), small.data(), m,
                           rtol, kRank3MaxIters, rx);
    }
    std::vector<uint16_t> tb(ne);
    for (long i = 0; i < ne; ++i) tb[i] = f32_to_bf16((float)tab[i]);
    return rank3_solve(tm, n, F, tb.data(), kinds, r, z, work.data(), tw.data(), small.data(), m,
                       rtol, kRank3MaxIters, RoundBf16());
}

// learned-setup judge of predicted factors Fp against SVD factors Fs (rank 2):
// out[0..4) = ||A - P(Fp)||_F, ||A - P(Fs)||_F, ||A||_F, guard estimate;
// returns 1 if accepted, 0 if not, -1 on a table failure
int kph_learned_judge(int dim, int n, const double* rec, const double* Fp, const double* Fs, double factor,
                      double guard, double* out) {
    Tables1D t;
    if (!make_tables(n, &t)) return -1;
    std::vector<double> tab(tab_entries(n));
    std::vector<int8_t> kinds(kMaxN);
    if (kph_form_tables(dim, n, 2, Fs, tab.data(), kinds.data()) != 0) return -1;
    HostTeam tm;
    std::vector<double> work(judge_work_doubles(dim, n));
    return learned_judge(tm, dim, n, t, rec, Fp, Fs, tab.data(), kinds.data(), work.data(), factor, guard, out)
               ? 1
               : 0;
}

// setup of one general (quadrature-data) element: factors [5 or 4][n][n],
// sigma[4]; returns the element status (or -1 for unsupported sizes)
int kph_setup_quad(int dim, int n, int mu, double tau, const double* c, const double* a, const double* nu,
                   const double* g, double* factors, double* sigma) {
    static QuadTables Q;
    if (!make_quad_tables(n, mu, &Q)) return -1;
    HostTeam tm;
    std::vector<double> work(quad_setup_doubles(dim, n, mu));
    QuadScratch qs;
    SetupWork W = carve_quad_setup(work.data(), n, &qs);
    QuadElem el{dim, n, mu, tau, c, a, nu, g};
    Term2 T2[kQuadGroups3];
    return setup_quad_element(tm, el, Q, factors, sigma, W, qs, T2);
}

// nc-component 2D system block (explicit, (m n)^2, m = nc n): factors
// [A1 m^2, B1 n^2, A2 m^2, B2 n^2], sigma[4], tables (sys_tab_entries) and
// kinds[n]; returns the status bits
int kph_sys_setup(int nc, int n, const double* block, double* F, double* sigma, double* tab, int8_t* kinds) {
    const int m = nc * n;
    if (m > kSysMaxM) return -1;
    HostTeam tm;
    std::vector<double> work(sys_work_doubles(m, n));
    double* tw = nullptr;
    SetupWork W = carve_sys(work.data(), m, n, &tw);
    double sh[kMaxN + 8];
    int st = setup_sys_element(tm, m, n, block, F, sigma, W);
    st |= tables_sys(tm, m, n, F, tab, kinds, tw, sh);
    return st;
}

// z = P^{-1} r for a system element (prec 0: FP64, 1: FP32 tables and arithmetic)
int kph_sys_apply(int nc, int n, int prec, const double* tab, const int8_t* kinds, const double* r, double* z) {
    const int m = nc * n;
    HostTeam tm;
    const long md = (long)m * n, ne = sys_tab_entries(m, n);
    if (prec == 0) {
        std::vector<double> X(r, r + md), Y(md), H(2 * m);
        apply_sys(tm, m, n, tab, kinds, X.data(), Y.data(), H.data());
        memcpy(z, X.data(), md * sizeof(double));
        return 0;
    }
    std::vector<float> tf(ne), X(md), Y(md), H(2 * m);
    for (long i = 0; i < ne; ++i) tf[i] = (float)tab[i];
    for (long i = 0; i < md; ++i) X[i] = (float)r[i];
    apply_sys(tm, m, n, tf.data(), kinds, X.data(), Y.data(), H.data());
    for (long i = 0; i < md; ++i) z[i] = X[i];
    return 0;
}

int kph_schur(int n, const double* C, double* T, double* Q) {
    HostTeam tm;
    double sh[kMaxN + 8];
    memcpy(T, C, n * n * sizeof(double));
    return real_schur(tm, n, T, Q, sh) ? 0 : 1;
}

}  // extern "C"
