"""1D nodal tables on the reference interval [0,1] (Sec. 3.1 and 3.2).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Nodal Lagrange basis on the n = p+1 Gauss-Legendre points of [0,1]
(Sec. 3.1); quadrature on the same points (collocation, mu = p+1, Sec. 3.1):
  W = diag(w),  D[a, j] = phi_j'(x_a)  (rows are quadrature points, Sec. 3.2),
  S = D^T W     (so u^T S v = int u' v),   K = D^T W D,
  l0[j] = phi_j(0),  l1[j] = phi_j(1).

Pinned by tests/test_oracle_tables.py (exactness of the rule, derivative of
monomials, summation by parts, K 1 = 0, the n^2 trace-inverse constant).
"""
from __future__ import annotations

import numpy as np


def gauss_legendre01(n: int):
    """Nodes and weights of the n-point Gauss-Legendre rule mapped to [0,1]."""
    xi, om = np.polynomial.legendre.leggauss(n)
    return 0.5 * (xi + 1.0), 0.5 * om


def lagrange_values(x: np.ndarray, t: float) -> np.ndarray:
    """phi_j(t) = prod_{k != j} (t - x_k) / (x_j - x_k), written out."""
    n = len(x)
    out = np.empty(n)
    for j in range(n):
        num = 1.0
        den = 1.0
        for k in range(n):
            if k != j:
                num *= t - x[k]
                den *= x[j] - x[k]
        out[j] = num / den
    return out


def lagrange_derivative_matrix(x: np.ndarray) -> np.ndarray:
    """D[a, j] = phi_j'(x_a) by the product rule.

    For a != j only the term that drops the factor (x - x_a) survives
    (phi_j vanishes at x_a); for a == j the derivative is sum_{m != j} 1/(x_j - x_m).
    """
    n = len(x)
    D = np.empty((n, n))
    for j in range(n):
        den = 1.0
        for k in range(n):
            if k != j:
                den *= x[j] - x[k]
        for a in range(n):
            if a == j:
                D[a, j] = sum(1.0 / (x[j] - x[m]) for m in range(n) if m != j)
            else:
                num = 1.0
                for k in range(n):
                    if k != j and k != a:
                        num *= x[a] - x[k]
                D[a, j] = num / den
    return D


def tables(n: int) -> dict:
    """All 1D tables for n nodes (Sec. 3.2, Table 1 with G = I)."""
    x, w = gauss_legendre01(n)
    W = np.diag(w)
    D = lagrange_derivative_matrix(x)
    S = D.T @ W
    K = D.T @ W @ D
    return dict(n=n, x=x, w=w, W=W, D=D, S=S, K=K,
                l0=lagrange_values(x, 0.0), l1=lagrange_values(x, 1.0))
