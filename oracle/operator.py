"""Global operator of the synthetic DG system: diagonal blocks plus upwind coupling.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The global matrix M - tau*J (Sec. 3.3) is block-structured: one diagonal block
per element (``oracle.blocks.element_block``) plus off-diagonal blocks that
couple neighbours through their common face (Sec. 3.3.1, the face part of
eq. jac-entries).  With the upwind flux and element-constant velocity
a = -beta, element e takes the neighbour's trace on every inflow face:
for axis k with beta_k < 0 the inflow face is the low face (l0) and the
neighbour is the low neighbour, whose trace is taken at its high face (l1);
for beta_k > 0 it is the high face (l1) and the high neighbour's low-face
trace (l0).  The off-diagonal block is
  -tau*|beta_k| * (l_in l_out^T on axis k) (x) W on the other axes.
Elements whose face flag is zero have no coupling (block-diagonal system).

Two forms: ``apply`` (matrix-free, dense per-element blocks) and
``assemble`` (scipy.sparse, small meshes).  Pinned by
tests/test_oracle_operator.py (the two forms agree; discrete conservation
1^T (G - mass) = 0 for a uniform velocity).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .blocks import element_block, kron_list
from .tables import tables


def coupling_block(rec: np.ndarray, ax: int, dim: int, T: dict):
    """(neighbour column index in the neighbour table, dense block) or None."""
    beta, tau = rec[ax], rec[6]
    if rec[7] == 0.0 or beta == 0.0:
        return None
    if beta < 0.0:
        l_in, l_out, col = T["l0"], T["l1"], 2 * ax
    else:
        l_in, l_out, col = T["l1"], T["l0"], 2 * ax + 1
    mats = [T["W"]] * dim
    mats[ax] = -tau * abs(beta) * np.outer(l_in, l_out)
    return col, kron_list(mats)


def apply(params: np.ndarray, nbr: np.ndarray, n: int, dim: int, x: np.ndarray,
          blocks: np.ndarray | None = None) -> np.ndarray:
    """y = G x for x of shape (E, n^d)."""
    T = tables(n)
    E = params.shape[0]
    y = np.empty_like(x)
    for e in range(E):
        A = blocks[e] if blocks is not None else element_block(params[e], n, dim, T)
        ye = A @ x[e]
        for ax in range(dim):
            cb = coupling_block(params[e], ax, dim, T)
            if cb is not None:
                col, C = cb
                ye = ye + C @ x[nbr[e, col]]
        y[e] = ye
    return y


def assemble(params: np.ndarray, nbr: np.ndarray, n: int, dim: int) -> sp.csr_matrix:
    T = tables(n)
    E = params.shape[0]
    N = n ** dim
    G = sp.lil_matrix((E * N, E * N))
    for e in range(E):
        G[e * N:(e + 1) * N, e * N:(e + 1) * N] = element_block(params[e], n, dim, T)
        for ax in range(dim):
            cb = coupling_block(params[e], ax, dim, T)
            if cb is not None:
                col, C = cb
                f = int(nbr[e, col])
                G[e * N:(e + 1) * N, f * N:(f + 1) * N] = (
                    G[e * N:(e + 1) * N, f * N:(f + 1) * N].toarray() + C)
    return G.tocsr()
