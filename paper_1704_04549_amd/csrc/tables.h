// 1D nodal tables on the reference interval [0,1] (Sec. 3.1-3.2).
//
// n Gauss-Legendre nodes x (ascending) and weights w; the Lagrange basis on
// those nodes; D[a*n + j] = phi_j'(x_a); S = D^T W; K = D^T W D;
// l0[j] = phi_j(0), l1[j] = phi_j(1).  Row-major n x n arrays.
#pragma once

#include "kp_common.h"

namespace kp {

struct Tables1D {
    int n;
    int pad;
    double x[kMaxN], w[kMaxN], l0[kMaxN], l1[kMaxN];
    double D[kMaxN * kMaxN], S[kMaxN * kMaxN], K[kMaxN * kMaxN];
};

// Fills t for 2 <= n <= kMaxN; returns false otherwise.
bool make_tables(int n, Tables1D* t);

}  // namespace kp
