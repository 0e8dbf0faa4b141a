"""Blocks of nc-component systems (Sec. 5.3: the Euler equations' blocks of
size nc (p+1)^2) and their KSVD with nc(p+1) x nc(p+1) first factors.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Nodal vectors are ordered (component, x, y), component slowest, so the first
Kronecker factor acts on the pair (component, x): the factorisation of the
paper's systems experiments, A ~ A1 (x) B1 + A2 (x) B2 with A_j of size
nc n x nc n and B_j of size n x n.

The 2D block of element k with flux Jacobians J_x, J_y (nc x nc, element
constant), the scalar mass coefficient c = 1 + alpha sin(pi x y + phi) at the
nodes and a second-order coefficient nu (the same weak form as the scalar
blocks, eq. adv-kron, with the advection velocity replaced by the Jacobian):

  A = I (x) diag(w (x) w * c)
      + tau [ -J_x (x) S (x) W - J_y (x) W (x) S + nu I (x) (K (x) W + W (x) K) ]
      + tau [ (J_x)^+ (x) l1 l1^T (x) W + (-J_x)^+ (x) l0 l0^T (x) W
              + (J_y)^+ (x) W (x) l1 l1^T + (-J_y)^+ (x) W (x) l0 l0^T ]   (faces)

with S = D^T W, K = D^T W D, l0/l1 the basis values at 0/1 and (X)^+ the
outflow part of the upwind flux Jacobian.  With nc = 1 and J_i = -beta_i it is
the scalar block of ``oracle.blocks`` (u_f = (J n)^+ on each face).

``small_blocks``: the nc diagonal component blocks (n^2 x n^2) of A, the
"small" block Jacobi variant of Sec. 5.6 that does not couple the components.

Pinned by tests/test_oracle_systems.py (nc = 1 reduction to the scalar block,
exact rank 2 with alpha = nu = 0 and no faces, Eckart-Young residual, the
dense solve of P).
"""
from __future__ import annotations

import numpy as np

from .ksvd import ksvd
from .tables import tables


def element_block(sysd: dict, e: int, n: int, T: dict | None = None) -> np.ndarray:
    if T is None:
        T = tables(n)
    nc, tau = sysd["nc"], sysd["tau"]
    w, W, S, K = T["w"], T["W"], T["S"], T["K"]
    x = T["x"]
    X, Y = np.meshgrid(x, x, indexing="ij")
    c = 1.0 + sysd["alpha"][e] * np.sin(np.pi * X * Y + sysd["phi"][e])
    I = np.eye(nc)
    A = np.kron(I, np.diag(np.kron(w, w) * c.ravel()))
    Jx, Jy = sysd["J"][e]
    nu = sysd["nu"][e]
    A = A + tau * (-np.kron(Jx, np.kron(S, W)) - np.kron(Jy, np.kron(W, S))
                   + nu * np.kron(I, np.kron(K, W) + np.kron(W, K)))
    if sysd["face"]:
        L0, L1 = np.outer(T["l0"], T["l0"]), np.outer(T["l1"], T["l1"])
        (Jpx, Jpy), (Jmx, Jmy) = sysd["Jp"][e], sysd["Jm"][e]
        A = A + tau * (np.kron(Jpx, np.kron(L1, W)) + np.kron(Jmx, np.kron(L0, W))
                       + np.kron(Jpy, np.kron(W, L1)) + np.kron(Jmy, np.kron(W, L0)))
    return A


def ksvd_system(A: np.ndarray, nc: int, n: int, r: int = 2) -> dict:
    """Best r-term sum of A_j (nc n x nc n) (x) B_j (n x n) by the full SVD of
    R(A) (Sec. 4.1 with m1 = n1 = nc n, m2 = n2 = n)."""
    m = nc * n
    s, As, Bs = ksvd(A, m, m, n, n, r)
    return dict(dim=2, n=n, nc=nc, rank=r, sigma=s, A=As, B=Bs)


def small_blocks(A: np.ndarray, nc: int, n: int) -> list:
    """The nc diagonal (component, component) blocks of A, n^2 x n^2 each."""
    N = n * n
    return [A[i * N:(i + 1) * N, i * N:(i + 1) * N] for i in range(nc)]
