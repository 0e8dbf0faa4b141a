"""Pins of the oracle's global operator, exact block Jacobi and FGMRES."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import operator
from oracle.blocks import element_block
from oracle.krylov import bj_factor, bj_solve, fgmres
from oracle.tables import tables


@pytest.mark.parametrize("dim,n,mesh", [(2, 4, 3), (3, 3, 2)])
def test_matrix_free_equals_assembled(dim, n, mesh):
    E = mesh ** dim
    params, nbr = synth.mesh_params(mesh, dim, seed=5)
    x = np.random.default_rng(0).standard_normal((E, n ** dim))
    y = operator.apply(params, nbr, n, dim, x)
    G = operator.assemble(params, nbr, n, dim)
    np.testing.assert_allclose(y.ravel(), G @ x.ravel(), atol=1e-13)


@pytest.mark.parametrize("dim,n,mesh", [(2, 5, 4), (3, 3, 3)])
def test_discrete_conservation_uniform_velocity(dim, n, mesh):
    # equal beta everywhere: volume terms have zero column sums and each outflow
    # self-term cancels the neighbour's inflow term, so 1^T (G - mass) = 0
    E = mesh ** dim
    params = np.repeat(synth.draw_params(1, dim, seed=8, face=True), E, axis=0)
    nbr = synth.periodic_neighbours(mesh, dim)
    G = operator.assemble(params, nbr, n, dim).toarray()
    T = tables(n)
    mass_rec = params[0].copy()
    mass_rec[6] = 0.0
    mass = np.kron(np.eye(E), element_block(mass_rec, n, dim, T))
    assert np.max(np.abs(np.ones(G.shape[0]) @ (G - mass))) < 1e-14 * np.abs(G).max() * n ** 2


def test_fgmres_one_step_with_exact_inverse():
    n, E = 6, 5
    params = synth.draw_params(E, 2, seed=2)
    T = tables(n)
    blocks = np.stack([element_block(r, n, 2, T) for r in params])
    lus = bj_factor(blocks)
    b = np.random.default_rng(3).standard_normal(E * n * n)
    Aop = lambda v: np.einsum("eij,ej->ei", blocks, v.reshape(E, -1)).ravel()
    Mop = lambda v: bj_solve(lus, v.reshape(E, -1)).ravel()
    x, it, hist, ok = fgmres(Aop, Mop, b, m=30, rtol=1e-10)
    assert ok and it == 1
    assert np.linalg.norm(Aop(x) - b) <= 1e-10 * np.linalg.norm(b)


def test_fgmres_matches_dense_solve_and_gmres_history():
    dim, n, mesh = 2, 4, 3
    E = mesh ** dim
    params, nbr = synth.mesh_params(mesh, dim, seed=6)
    G = operator.assemble(params, nbr, n, dim).toarray()
    T = tables(n)
    blocks = np.stack([element_block(r, n, dim, T) for r in params])
    lus = bj_factor(blocks)
    b = np.random.default_rng(4).standard_normal(G.shape[0])
    Mop = lambda v: bj_solve(lus, v.reshape(E, -1)).ravel()
    x, it, hist, ok = fgmres(lambda v: G @ v, Mop, b, m=10, rtol=1e-10)
    assert ok
    np.testing.assert_allclose(x, np.linalg.solve(G, b), rtol=0, atol=1e-8 * np.abs(x).max())
    # with a fixed linear M, FGMRES is right-preconditioned GMRES: same residual history
    AM = spla.LinearOperator(G.shape, matvec=lambda v: G @ Mop(v))
    ref = []
    spla.gmres(AM, b, rtol=1e-10, restart=10, maxiter=50, callback=lambda r: ref.append(r),
               callback_type="pr_norm")
    k = min(len(ref), 10)
    np.testing.assert_allclose(hist[:k], ref[:k], rtol=1e-6)
