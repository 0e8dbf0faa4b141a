// Host construction of the 1D tables (Sec. 3.1-3.2).
//
// Gauss-Legendre nodes by Newton's method on the Legendre polynomial P_n
// (three-term recurrence, derivative n (x P_n - P_{n-1}) / (x^2 - 1)) from the
// usual cosine initial guesses; weights 2 / ((1 - x^2) P_n'(x)^2).  The
// differentiation matrix and boundary values use the barycentric form of the
// Lagrange basis (weights lambda_j = 1 / prod_{k != j}(x_j - x_k)).
#include "tables.h"

#include <string.h>

namespace kp {

static void legendre(int n, double z, double* pn, double* dpn) {
    double p0 = 1.0, p1 = z;
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    *pn = p1;
    *dpn = n * (z * p1 - p0) / (z * z - 1.0);
}

bool make_tables(int n, Tables1D* t) {
    if (n < 2 || n > kMaxN) return false;
    memset(t, 0, sizeof(*t));
    t->n = n;
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double z = cos(pi * (i + 0.75) / (n + 0.5));  // descending roots
        double pn = 0, dpn = 1;
        for (int it = 0; it < 100; ++it) {
            legendre(n, z, &pn, &dpn);
            double dz = pn / dpn;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        legendre(n, z, &pn, &dpn);
        t->x[i] = 0.5 * (1.0 - z);                  // ascending on [0,1]
        t->w[i] = 1.0 / ((1.0 - z * z) * dpn * dpn);  // (2 / ...) / 2
    }
    double lam[kMaxN];
    for (int j = 0; j < n; ++j) {
        double p = 1.0;
        for (int k = 0; k < n; ++k)
            if (k != j) p *= (t->x[j] - t->x[k]);
        lam[j] = 1.0 / p;
    }
    for (int a = 0; a < n; ++a) {
        double diag = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == a) continue;
            double v = (lam[j] / lam[a]) / (t->x[a] - t->x[j]);
            t->D[a * n + j] = v;
            diag -= v;
        }
        t->D[a * n + a] = diag;
    }
    for (int e = 0; e < 2; ++e) {
        double s = (double)e, den = 0.0;
        double* l = e ? t->l1 : t->l0;
        for (int j = 0; j < n; ++j) den += lam[j] / (s - t->x[j]);
        for (int j = 0; j < n; ++j) l[j] = (lam[j] / (s - t->x[j])) / den;
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            t->S[i * n + j] = t->D[j * n + i] * t->w[j];
            double k = 0.0;
            for (int a = 0; a < n; ++a) k += t->D[a * n + i] * t->w[a] * t->D[a * n + j];
            t->K[i * n + j] = k;
        }
    return true;
}

}  // namespace kp
