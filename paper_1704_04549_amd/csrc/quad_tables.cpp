// Host construction of the tables of a general element's (n, mu) pair
// (Sec. 3.1, Sec. 3.4.1): the mu-point Gauss-Legendre rule of [0,1], the
// Lagrange basis on the n Gauss-Legendre nodes and its derivative at those
// points (product rule: phi_j'(x) = sum_{m != j} prod_{k != j, m} (x - x_k) /
// prod_{k != j} (x_j - x_k)), phi(0), phi(1), and the Grams of the pair types.
#include <string.h>

#include "quad.h"
#include "tables.h"

namespace kp {

bool make_quad_tables(int n, int mu, QuadTables* Q) {
    if (n < 2 || n > kMaxN || mu < n || mu > kQuadMaxMu) return false;
    Tables1D tn, tm;
    if (!make_tables(n, &tn) || !make_tables(mu, &tm)) return false;
    memset(Q, 0, sizeof(*Q));
    Q->n = n;
    Q->mu = mu;
    const double* x = tn.x;
    for (int al = 0; al < mu; ++al) {
        Q->w[al] = tm.w[al];
        const double t = tm.x[al];
        for (int j = 0; j < n; ++j) {
            double den = 1.0, val = 1.0;
            for (int k = 0; k < n; ++k)
                if (k != j) {
                    den *= x[j] - x[k];
                    val *= t - x[k];
                }
            double der = 0.0;
            for (int m = 0; m < n; ++m) {
                if (m == j) continue;
                double p = 1.0;
                for (int k = 0; k < n; ++k)
                    if (k != j && k != m) p *= t - x[k];
                der += p;
            }
            Q->Phi[al * n + j] = val / den;
            Q->dPhi[al * n + j] = der / den;
        }
    }
    for (int j = 0; j < n; ++j) {
        Q->l0[j] = tn.l0[j];
        Q->l1[j] = tn.l1[j];
    }
    // K[p][q][a][b] = (L_p L_q^T)[a,b] (R_p R_q^T)[a,b]
    for (int p = 0; p < kQuadTypes; ++p)
        for (int q = 0; q < kQuadTypes; ++q)
            for (int a = 0; a < qmu(*Q, p); ++a)
                for (int b = 0; b < qmu(*Q, q); ++b) {
                    double sl = 0.0, sr = 0.0;
                    for (int i = 0; i < n; ++i) {
                        sl += qL(*Q, p, a, i) * qL(*Q, q, b, i);
                        sr += qR(*Q, p, a, i) * qR(*Q, q, b, i);
                    }
                    Q->K[(p * kQuadTypes + q) * kQuadMaxMu * kQuadMaxMu + a * kQuadMaxMu + b] = sl * sr;
                }
    return true;
}

}  // namespace kp
