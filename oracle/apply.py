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
quasi-triangular solve is Bartels-Stewart: blocks of Y are solved from the
bottom-right corner, each a system of size at most 4 (a 2x2 diagonal block of
T1 or T2 couples two rows or two columns), after O(n) updates per unknown.

``Flops`` counts the operations of the fast path, to check the operation
counts of Sec. 4.4 (O(p^3) per 2D apply, O(p^4) per 3D apply).

``eig_fdm_solve``: fast diagonalisation with the (complex) eigendecomposition,
the alternative the paper mentions in Sec. 4.2; used only as a pin on
small n.

Pinned by tests/test_oracle_apply.py (P z = r residual, Schur = dense,
FDM = dense on n <= 6, hand-written Sylvester = scipy.linalg.solve_sylvester)
and tests/test_oracle_shuffled.py (operation counts against 14 n^3 / 16 n^4
and their growth rates in n).
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


class Flops:
    """Operation counter of the fast CPU path: every counted helper below adds
    the floating-point operations of the operation it performs (one add, one
    multiply or one divide each), from the shapes of its actual operands."""

    def __init__(self):
        self.count = 0

    def add(self, k: int) -> None:
        self.count += int(k)


def _mm(A: np.ndarray, B: np.ndarray, fc: Flops | None) -> np.ndarray:
    """A @ B (batched over leading axes): (2k - 1) operations per output entry,
    k the contracted length."""
    out = A @ B
    if fc is not None:
        fc.add(out.size * (2 * A.shape[-1] - 1))
    return out


def _lus(lu, B: np.ndarray, fc: Flops | None, trans: int = 0) -> np.ndarray:
    """LU solve with k right-hand sides: unit-lower forward substitution
    n (n - 1) and upper back substitution n^2 operations per right-hand side."""
    if fc is not None:
        n = lu[0].shape[0]
        k = B.shape[1] if B.ndim == 2 else 1
        fc.add(k * (2 * n * n - n))
    return sla.lu_solve(lu, B, trans=trans)


def _blocks(T: np.ndarray):
    """Diagonal blocks (start, size) of an upper quasi-triangular matrix, last first."""
    n = T.shape[0]
    out = []
    j = n - 1
    while j >= 0:
        if j > 0 and T[j, j - 1] != 0.0:
            out.append((j - 1, 2))
            j -= 2
        else:
            out.append((j, 1))
            j -= 1
    return out


def quasi_tri_sylvester(T1: np.ndarray, T2: np.ndarray, F: np.ndarray, fc: Flops | None = None) -> np.ndarray:
    """Solve T1 Y + Y T2^T = F for upper quasi-triangular T1, T2 (Bartels-Stewart).

    F may carry leading batch axes (independent systems with the same T1, T2).
    Column blocks J of Y (the 1x1 and 2x2 diagonal blocks of T2) go from last
    to first; within one, row blocks I (those of T1) from last to first.  Each
    (I, J) block solves the small system T1_II Y_IJ + Y_IJ T2_JJ^T = G_IJ of
    size at most 4, after the updates by the blocks already solved:
      G_IJ = F_IJ - sum_{K > J} Y_IK T2_JK^T - sum_{M > I} T1_IM Y_MJ.
    O(n^3) operations per system: each of the n^2 unknowns takes O(n) updates."""
    n = T1.shape[0]
    Y = np.zeros_like(F)
    nb = F.size // (n * n)
    rows = _blocks(T1)
    for j0, sj in _blocks(T2):
        J = slice(j0, j0 + sj)
        # the column block's right-hand side after the solved columns
        G = F[..., :, J].copy()
        if j0 + sj < n:
            G -= _mm(Y[..., :, j0 + sj:], T2[J, j0 + sj:].T, fc)
            if fc is not None:
                fc.add(nb * n * sj)
        for i0, si in rows:
            I = slice(i0, i0 + si)
            g = G[..., I, :].copy()
            if i0 + si < n:
                g -= _mm(T1[I, i0 + si:], Y[..., i0 + si:, J], fc)
                if fc is not None:
                    fc.add(nb * si * sj)
            # (I_sj (x) T1_II + T2_JJ (x) I_si) vec_col(Y_IJ) = vec_col(g)
            K = np.kron(np.eye(sj), T1[I, I]) + np.kron(T2[J, J], np.eye(si))
            m = si * sj
            if fc is not None:
                fc.add(nb * (2 * m * m - m) + (2 * m ** 3) // 3)
            rhs = np.swapaxes(g, -1, -2).reshape(-1, m).T          # columns: vec_col(g) per system
            sol = np.linalg.solve(K, rhs).T.reshape(g.shape[:-2] + (sj, si))
            Y[..., I, J] = np.swapaxes(sol, -1, -2)
    return Y


class SchurPrecond:
    """Alg. 5/7 (form) and Alg. 6/8 (apply) on the CPU in FP64.

    ``solve(r, fc)`` counts its operations in ``fc`` (a ``Flops``) when one is
    given: the fast path of Algs. 6/8 costs about 14 n^3 (2D: two inverse
    factors 4 n^3, Q^T 4 n^3, Sylvester 2 n^3, Q 4 n^3) and 16 n^4 (3D: three
    inverse factors 6 n^4, Q^T 4 n^4, n Sylvester solves 2 n^4, Q 4 n^4)
    operations, i.e. O(p^{d+1}) (Sec. 4.4)."""

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

    def _sylv(self, Rt: np.ndarray, fc: Flops | None) -> np.ndarray:
        F = _mm(_mm(self.Q1.T, Rt, fc), self.Q2, fc)
        Y = quasi_tri_sylvester(self.T1, self.T2, F, fc)
        return _mm(_mm(self.Q1, Y, fc), self.Q2.T, fc)

    def solve(self, r: np.ndarray, fc: Flops | None = None) -> np.ndarray:
        n = self.n
        if self.dim == 2:
            R = r.reshape(n, n)
            Rt = _lus(self.lu_x, R, fc)
            Rt = _lus(self.lu_y, Rt.T, fc).T
            return self._sylv(Rt, fc).reshape(-1)
        R = r.reshape(n, n, n)
        R = _lus(self.lu_x, R.reshape(n, n * n), fc).reshape(n, n, n)
        R = np.stack([_lus(self.lu_y, R[a], fc) for a in range(n)])
        R = np.stack([_lus(self.lu_z, R[a].T, fc).T for a in range(n)])
        return self._sylv(R, fc).reshape(-1)   # the n slices' systems together


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
