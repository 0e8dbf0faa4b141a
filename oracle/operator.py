"""Global operator of the synthetic DG system: diagonal blocks plus upwind coupling.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The global matrix M - tau*J (Sec. 3.4) is block-structured: one diagonal block
per element (``oracle.blocks.element_block``) plus off-diagonal blocks that
couple neighbours through their common face (Sec. 3.4.1, the face part of
eq. jac-entries).  The upwind flux on each face uses one normal velocity u_f
(record entries 8..13; u_f > 0 is outflow).  On an inflow face (u_f < 0) the
element takes the neighbour's trace: the off-diagonal block is
  tau*u_f * (l_face l_opp^T on the face's axis) (x) W on the other axes,
with l_face = l0 (low face) or l1 (high face) and l_opp the neighbour's
opposite face (l1 or l0).  Elements whose face flag is zero have no coupling.

Two forms: ``apply`` (matrix-free, dense per-element blocks) and
``assemble`` (scipy.sparse, small meshes).  Pinned by
tests/test_oracle_operator_krylov.py (the two forms agree; discrete
conservation 1^T (G - mass) = 0 for a uniform velocity; every coupling block
equals the upwind face integral of the weak form on polynomials, which fixes
its sign, face pairing and neighbour side).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .blocks import element_block, kron_list
from .tables import tables


def coupling_blocks(rec: np.ndarray, ax: int, dim: int, T: dict):
    """[(neighbour column index in the neighbour table, dense block)] for one axis."""
    out = []
    if rec[7] == 0.0:
        return out
    tau = rec[6]
    for side, l_in, l_out in ((0, T["l0"], T["l1"]), (1, T["l1"], T["l0"])):
        u = rec[8 + 2 * ax + side]
        if u < 0.0:
            mats = [T["W"]] * dim
            mats[ax] = tau * u * np.outer(l_in, l_out)
            out.append((2 * ax + side, kron_list(mats)))
    return out


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
            for col, C in coupling_blocks(params[e], ax, dim, T):
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
            for col, C in coupling_blocks(params[e], ax, dim, T):
                f = int(nbr[e, col])
                G[e * N:(e + 1) * N, f * N:(f + 1) * N] = (
                    G[e * N:(e + 1) * N, f * N:(f + 1) * N].toarray() + C)
    return G.tocsr()
