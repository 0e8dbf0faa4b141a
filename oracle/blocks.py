"""Explicit element blocks A_k of M - tau*J for the synthetic DG operator.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The block is the collocated (G = I) tensor-product form of the implicit
system's diagonal block (Sec. 3.4, implicit time integration; Table 1; the
advection Kronecker form of Sec. 5.1, eq. adv-kron), for the scalar problem
with element-constant velocity a = -beta, a diffusion-like term nu*K and a
point-wise mass coefficient c:

  2D: A = diag(w(x)w * c) + tau*[beta_x S(x)W + beta_y W(x)S + nu (K(x)W + W(x)K)]
  3D: A = diag(w(x)w(x)w * c) + tau*[beta_x S(x)W(x)W + beta_y W(x)S(x)W
          + beta_z W(x)W(x)S + nu (K(x)W(x)W + W(x)K(x)W + W(x)W(x)K)]

with c(x_i, y_j[, z_k]) = 1 + alpha sin(pi x_i y_j [z_k] + phi) at the nodes of
the reference element [0,1]^d.  The first Kronecker factor is the x axis, the
slowest index of the nodal vector: u[(i*n + j)*n + k].

With the record's face flag set, the outflow self-terms of the upwind flux are
added to the block (weak form, eq. weak-form; the face part of eq.
jac-entries).  The numerical flux on a face uses one normal velocity u_f
(record entries 8..13 for the faces x-, x+, y-, y+, z-, z+; u_f > 0 is
outflow).  An outflow face contributes tau*u_f * (l l^T) on its axis times W on
the other axes, with l = l0 on the low face and l1 on the high face.

Pinned by tests/test_oracle_blocks.py (the bilinear form against an
independent higher-order quadrature of the weak form, alpha = 0 separability).
"""
from __future__ import annotations

import numpy as np

from .tables import tables


def coefficient(rec: np.ndarray, x: np.ndarray, dim: int) -> np.ndarray:
    """c at the tensor nodes, flattened in nodal order."""
    alpha, phi = rec[4], rec[5]
    if dim == 2:
        X, Y = np.meshgrid(x, x, indexing="ij")
        prod = X * Y
    else:
        X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
        prod = X * Y * Z
    return (1.0 + alpha * np.sin(np.pi * prod + phi)).ravel()


def axis_operator(rec: np.ndarray, ax: int, T: dict) -> np.ndarray:
    """1D part of the block along one axis: tau*(beta S + nu K) + outflow face terms."""
    beta, nu, tau = rec[ax], rec[3], rec[6]
    X = tau * (beta * T["S"] + nu * T["K"])
    if rec[7] != 0.0:
        for side, l in ((0, T["l0"]), (1, T["l1"])):
            u = rec[8 + 2 * ax + side]
            if u > 0.0:
                X = X + tau * u * np.outer(l, l)
    return X


def kron_list(mats):
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(out, m)
    return out


def element_block(rec: np.ndarray, n: int, dim: int, T: dict | None = None) -> np.ndarray:
    """Dense n^d x n^d block of one element."""
    if T is None:
        T = tables(n)
    w, W = T["w"], T["W"]
    mass = kron_list([w] * dim) * coefficient(rec, T["x"], dim)
    A = np.diag(mass)
    for ax in range(dim):
        mats = [W] * dim
        mats[ax] = axis_operator(rec, ax, T)
        A = A + kron_list(mats)
    return A


def element_blocks(params: np.ndarray, n: int, dim: int) -> np.ndarray:
    T = tables(n)
    return np.stack([element_block(r, n, dim, T) for r in params])
