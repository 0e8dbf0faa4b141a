// Host build of the per-element routines under AddressSanitizer: every table,
// vector and coefficient array an element's routine reads is a heap buffer of
// exactly the size the kernels' layout gives it, so an index outside the
// element's data (a table row past the last N_j, a lane index >= n, a face
// array past its end) is reported.  Covers table formation and the generic
// apply for 2D n = 2..32 and 3D n = 2..16 in FP64, FP32 and split BF16, the
// structured setup, the learned-setup judge, the general-element setup, and
// the systems blocks' setup, tables and apply (FP64, FP32).
// Built and run by tests/test_bounds_asan.py (CPU only).
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "elem_ops.h"
#include "learned.h"
#include "quad.h"
#include "sys.h"
#include "tables.h"

using namespace kp;

template <class T>
static T* exact(size_t count) {
    return (T*)malloc(count * sizeof(T) + (count == 0));
}

int main() {
    std::mt19937_64 rng(7);
    std::normal_distribution<double> nd01(0.0, 1.0);
    std::uniform_real_distribution<double> u01(0.0, 1.0);
    HostTeam tm;
    int checked = 0;
    for (int dim = 2; dim <= 3; ++dim)
        for (int n = 2; n <= (dim == 2 ? 32 : 16); ++n) {
            Tables1D T;
            if (!make_tables(n, &T)) return 2;
            const long nn = (long)n * n, nd = dim == 2 ? nn : nn * n;
            const int nf = dim == 2 ? 4 : 5;
            // a record with faces, and its structured setup
            double rec[kRecLen] = {};
            for (int i = 0; i < 3; ++i) rec[i] = 2.0 * u01(rng) - 1.0;
            rec[3] = 0.01;
            rec[4] = 0.3;
            rec[5] = 1.0;
            rec[6] = 0.1;
            rec[7] = 1.0;
            for (int f = 0; f < 6; ++f) rec[8 + f] = (f % 2 ? 1.0 : -1.0) * rec[f / 2];
            std::vector<double> ws(setup_work_doubles(dim, n, false, 2));
            SetupWork W = carve_setup_work(ws.data(), dim, n, false, 2);
            double* F = exact<double>(nf * nn);
            double* sig = exact<double>(4);
            setup_element<false>(tm, dim, n, 2, T, rec, nullptr, nullptr, F, sig, W);
            // tables and the apply in three precisions
            const long ne = tab_entries(n);
            double* tab = exact<double>(ne);
            int8_t* kinds = exact<int8_t>(kMaxN);
            double* wk = exact<double>(10 * nn + 64);
            int* piv = exact<int>(n + 1);
            double sh[kMaxN + 8];
            form_tables(tm, dim, n, 2, F, tab, tab + 7 * nn, kinds, wk, piv, sh);
            const long ns = dim == 2 ? 1 : n;
            double* X = exact<double>(nd);
            double* Y = exact<double>(nd);
            double* H = exact<double>(2 * n * ns);
            for (long t = 0; t < nd; ++t) X[t] = nd01(rng);
            apply_tensor(tm, dim, n, tab, kinds, X, Y, H, RoundNone());
            float* tf = exact<float>(ne);
            float* Xf = exact<float>(nd);
            float* Yf = exact<float>(nd);
            float* Hf = exact<float>(2 * n * ns);
            for (long t = 0; t < ne; ++t) tf[t] = (float)tab[t];
            for (long t = 0; t < nd; ++t) Xf[t] = (float)X[t];
            apply_tensor(tm, dim, n, tf, kinds, Xf, Yf, Hf, RoundNone());
            apply_tensor(tm, dim, n, tf, kinds, Xf, Yf, Hf, RoundBf16x2());
            uint16_t* tb = exact<uint16_t>(ne);
            for (long t = 0; t < ne; ++t) tb[t] = f32_to_bf16(tf[t]);
            apply_tensor(tm, dim, n, tb, kinds, Xf, Yf, Hf, RoundBf16());
            // the learned-setup judge (rank 2) on the element's own factors
            if (judge_work_doubles(dim, n) > 0) {
                double* jw = exact<double>(judge_work_doubles(dim, n));
                double out[4];
                learned_judge(tm, dim, n, T, rec, F, F, tab, kinds, jw, 1.1, 0.01, out);
                free(jw);
            }
            free(F); free(sig); free(tab); free(kinds); free(wk); free(piv); free(X); free(Y); free(H);
            free(tf); free(Xf); free(Yf); free(Hf); free(tb);
            ++checked;
        }
    // general elements
    static QuadTables Q;
    const int cases[][3] = {{2, 3, 3}, {2, 5, 8}, {2, 16, 17}, {2, 32, 32}, {3, 2, 2}, {3, 4, 6}, {3, 8, 9}, {3, 16, 17}};
    for (const auto& cs : cases) {
        const int dim = cs[0], n = cs[1], mu = cs[2];
        if (!make_quad_tables(n, mu, &Q)) return 3;
        const long md = dim == 2 ? (long)mu * mu : (long)mu * mu * mu, mf = dim == 2 ? mu : (long)mu * mu;
        double* c = exact<double>(md);
        double* a = exact<double>(dim * md);
        double* nu = exact<double>(md);
        double* g = exact<double>(2 * dim * mf);
        for (long t = 0; t < md; ++t) {
            c[t] = 1.0 + 0.1 * u01(rng);
            nu[t] = 0.01;
        }
        for (long t = 0; t < dim * md; ++t) a[t] = nd01(rng);
        for (long t = 0; t < 2 * dim * mf; ++t) g[t] = u01(rng);
        double* ws = exact<double>(quad_setup_doubles(dim, n, mu));
        QuadScratch qs;
        SetupWork W = carve_quad_setup(ws, n, &qs);
        const long nn = (long)n * n;
        double* F = exact<double>((dim == 2 ? 4 : 5) * nn);
        double* sig = exact<double>(4);
        QuadElem el{dim, n, mu, 0.1, c, a, nu, g};
        Term2 T2[kQuadGroups3];
        setup_quad_element(tm, el, Q, F, sig, W, qs, T2);
        free(c); free(a); free(nu); free(g); free(F); free(sig); free(ws);
        ++checked;
    }
    // systems blocks: nc components, m = nc n first factors
    const int scases[][2] = {{1, 2}, {2, 4}, {4, 4}, {3, 8}, {4, 8}, {2, 16}};
    for (const auto& cs : scases) {
        const int nc = cs[0], n = cs[1], m = nc * n;
        const long N = (long)m * n, md = N;
        double* A = exact<double>(N * N);
        for (long t = 0; t < N * N; ++t) A[t] = 0.05 * nd01(rng) + ((t / N == t % N) ? 2.0 : 0.0);
        double* ws = exact<double>(sys_work_doubles(m, n));
        double* tw = nullptr;
        SetupWork W = carve_sys(ws, m, n, &tw);
        double* F = exact<double>(sys_factor_entries(m, n));
        double* sig = exact<double>(4);
        const long ne = sys_tab_entries(m, n);
        double* tab = exact<double>(ne);
        int8_t* kinds = exact<int8_t>(kMaxN);
        double sh[kMaxN + 8];
        setup_sys_element(tm, m, n, A, F, sig, W);
        tables_sys(tm, m, n, F, tab, kinds, tw, sh);
        double* X = exact<double>(md);
        double* Y = exact<double>(md);
        double* H = exact<double>(2 * m);
        for (long t = 0; t < md; ++t) X[t] = nd01(rng);
        apply_sys(tm, m, n, tab, kinds, X, Y, H);
        float* tf = exact<float>(ne);
        float* Xf = exact<float>(md);
        float* Yf = exact<float>(md);
        float* Hf = exact<float>(2 * m);
        for (long t = 0; t < ne; ++t) tf[t] = (float)tab[t];
        for (long t = 0; t < md; ++t) Xf[t] = (float)nd01(rng);
        apply_sys(tm, m, n, tf, kinds, Xf, Yf, Hf);
        free(A); free(ws); free(F); free(sig); free(tab); free(kinds); free(X); free(Y); free(H);
        free(tf); free(Xf); free(Yf); free(Hf);
        ++checked;
    }
    printf("checked %d cases\n", checked);
    return 0;
}
