"""Applying the inverse of the Kronecker-sum preconditioner.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

``dense_solve``: the plain definition z = P^{-1} r with P assembled densely
from its factors and solved by LAPACK LU (eqs. 2d-kron-sum, 3d-simple-precond).
This is the reference every other apply is compared against.

``SchurPrecond``: the paper's own fast route, written from Sec. 4.2 (eq.
quad-triang) and Sec. 4.3 and Algs. 5-8.
  2D: multiply P x = b by A2^{-1} (x) B1^{-1}:
      (C1 (x) I + I (x) C2) x = (A2^{-1} (x) B1^{-1}) b, C1 = A2^{-1}A1, C2 = B1^{-1}B2;
      real Schur C_i = Q_i T_i Q_i^T; solve the quasi-triangular Sylvester system;
      x = (Q1 (x) Q2) x~.
  3D: multiply by A1^{-1} (x) B2^{-1} (x) C1^{-1}:
      (I (x) B2^{-1}B1 (x) I + I (x) I (x) C1^{-1}C2) x = (...) b, then the same
      Sylvester solve on every slice of the first index.
In matrix form, with X[i, j] = x[i*n + j], (C1 (x) I + I (x) C2) x is
C1 X + X C2^T, so each Sylvester system reads T1 Y + Y T2^T = F.  The
quasi-triangular solve sweeps the columns of Y from last to first; a 2x2
diagonal block of T2 couples two columns, which are then solved together
as one dense 2n x 2n system.

``eig_fdm_solve``: fast diagonalisation with the (complex) eigendecomposition,
the alternative the paper mentions in Sec. 4.2; used only as a pin on
small n.

Pinned by tests/test_oracle_apply.py (P z = r residual, Schur = dense,
FDM = dense on n <= 6, hand-written Sylvester = scipy.linalg.solve_sylvester).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .ksvd import precond_matrix


def dense_solve(f: dict, r: np.ndarray) -> np.ndarray:
    """z = P^{-1} r for r of shape (..., n^d) by dense LU of P."""
    P = precond_matrix(f)
    lu = sla.lu_factor(P)
    rr = np.asarray(r, dtype=np.float64)
    flat = rr.reshape(-1, P.shape[0]).T
    return sla.lu_solve(lu, flat).T.reshape(rr.shape)


def quasi_tri_sylvester(T1: np.ndarray, T2: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Solve T1 Y + Y T2^T = F for upper quasi-triangular T1, T2."""
    n = T1.shape[0]
    Y = np.zeros_like(F)
    I = np.eye(n)
    j = n - 1
    while j >= 0:
        pair = j > 0 and T2[j, j - 1] != 0.0
        if not pair:
            g = F[:, j] - Y[:, j + 1:] @ T2[j, j + 1:]
            Y[:, j] = np.linalg.solve(T1 + T2[j, j] * I, g)
            j -= 1
        else:
            i = j - 1
            gi = F[:, i] - Y[:, j + 1:] @ T2[i, j + 1:]
            gj = F[:, j] - Y[:, j + 1:] @ T2[j, j + 1:]
            M = np.block([[T1 + T2[i, i] * I, T2[i, j] * I],
                          [T2[j, i] * I, T1 + T2[j, j] * I]])
            y = np.linalg.solve(M, np.concatenate([gi, gj]))
            Y[:, i] = y[:n]
            Y[:, j] = y[n:]
            j -= 2
    return Y


class SchurPrecond:
    """Alg. 5/7 (form) and Alg. 6/8 (apply) on the CPU in FP64."""

    def __init__(self, f: dict):
        self.dim = f["dim"]
        self.n = f["n"]
        if self.dim == 2:
            assert f["rank"] == 2
            A1, A2 = f["A"]
            B1, B2 = f["B"]
            self.lu_x = sla.lu_factor(A2)
            self.lu_y = sla.lu_factor(B1)
            C1 = sla.lu_solve(self.lu_x, A1)
            C2 = sla.lu_solve(self.lu_y, B2)
        else:
            A1 = f["A1"]
            B1, B2 = f["B"]
            C1f, C2f = f["C"]
            self.lu_x = sla.lu_factor(A1)
            self.lu_y = sla.lu_factor(B2)
            self.lu_z = sla.lu_factor(C1f)
            C1 = sla.lu_solve(self.lu_y, B1)
            C2 = sla.lu_solve(self.lu_z, C2f)
        self.T1, self.Q1 = sla.schur(C1, output="real")
        self.T2, self.Q2 = sla.schur(C2, output="real")

    def _sylv(self, Rt: np.ndarray) -> np.ndarray:
        F = self.Q1.T @ Rt @ self.Q2
        Y = quasi_tri_sylvester(self.T1, self.T2, F)
        return self.Q1 @ Y @ self.Q2.T

    def solve(self, r: np.ndarray) -> np.ndarray:
        n = self.n
        if self.dim == 2:
            R = r.reshape(n, n)
            Rt = sla.lu_solve(self.lu_x, R)
            Rt = sla.lu_solve(self.lu_y, Rt.T).T
            return self._sylv(Rt).reshape(-1)
        R = r.reshape(n, n, n)
        R = sla.lu_solve(self.lu_x, R.reshape(n, n * n)).reshape(n, n, n)
        R = np.stack([sla.lu_solve(self.lu_y, R[a]) for a in range(n)])
        R = np.stack([sla.lu_solve(self.lu_z, R[a].T).T for a in range(n)])
        X = np.stack([self._sylv(R[a]) for a in range(n)])
        return X.reshape(-1)


def schur_solve(f: dict, r: np.ndarray) -> np.ndarray:
    pc = SchurPrecond(f)
    rr = np.asarray(r, dtype=np.float64)
    flat = rr.reshape(-1, f["n"] ** f["dim"])
    return np.stack([pc.solve(v) for v in flat]).reshape(rr.shape)


def eig_fdm_solve(f: dict, r: np.ndarray) -> np.ndarray:
    """2D fast diagonalisation through eigendecompositions of C1 and C2."""
    assert f["dim"] == 2 and f["rank"] == 2
    n = f["n"]
    A1, A2 = f["A"]
    B1, B2 = f["B"]
    C1 = np.linalg.solve(A2, A1)
    C2 = np.linalg.solve(B1, B2)
    l1, V1 = np.linalg.eig(C1)
    l2, V2 = np.linalg.eig(C2)
    R = r.reshape(n, n)
    Rt = np.linalg.solve(A2, R)
    Rt = np.linalg.solve(B1, Rt.T).T
    G = np.linalg.solve(V1, Rt)
    G = np.linalg.solve(V2, G.T).T
    Y = G / (l1[:, None] + l2[None, :])
    X = V1 @ Y @ V2.T
    return np.real(X).reshape(-1)
