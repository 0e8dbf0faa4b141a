"""Exact block Jacobi and flexible GMRES.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Exact block Jacobi: LU with partial pivoting of every diagonal block, z = A_k^{-1} r
(the comparator of Sec. 5; its O(p^{3d}) form cost is the point of the paper).

FGMRES(m): restarted GMRES with right preconditioning allowed to vary per
step (Saad's flexible variant; the paper solves with restarted preconditioned
GMRES, Sec. 5 opening).  x0 = 0; z_j = M(v_j); w = A z_j; modified Gram-Schmidt;
Givens rotations on the Hessenberg matrix; the cycle stops when the Givens
residual estimate is <= rtol*||b||; the restart then recomputes the true
residual b - A x and the solve ends once it is <= rtol*||b||.  The iteration
count is the total number of Arnoldi steps.

Pinned by tests/test_oracle_krylov.py (one step with M = A^{-1}; agreement with
a dense solve; the residual history equals that of GMRES on A M^{-1} for a
fixed linear M).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def bj_factor(blocks: np.ndarray):
    return [sla.lu_factor(A) for A in blocks]


def bj_solve(lus, r: np.ndarray) -> np.ndarray:
    """r of shape (E, N) or (E, nrhs, N)."""
    out = np.empty_like(r)
    for e, lu in enumerate(lus):
        if r.ndim == 2:
            out[e] = sla.lu_solve(lu, r[e])
        else:
            out[e] = sla.lu_solve(lu, r[e].T).T
    return out


def fgmres(Aop, Mop, b: np.ndarray, m: int = 30, rtol: float = 1e-10,
           maxit: int = 3000):
    """Returns (x, iterations, relative residual history, converged)."""
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    if nb == 0.0:
        return x, 0, [], True
    r = b.copy()
    beta = nb
    iters = 0
    hist = []
    while True:
        V = np.zeros((m + 1, b.size))
        Z = np.zeros((m, b.size))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = np.asarray(Mop(V[j])).ravel()
            w = np.asarray(Aop(Z[j])).ravel()
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            iters += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / nb)
            if abs(g[j + 1]) <= rtol * nb or iters >= maxit:
                break
        y = sla.solve_triangular(H[:k, :k], g[:k])
        x = x + Z[:k].T @ y
        r = b - np.asarray(Aop(x)).ravel()
        beta = np.linalg.norm(r)
        if beta <= rtol * nb:
            return x, iters, hist, True
        if iters >= maxit:
            return x, iters, hist, False
