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


@pytest.mark.parametrize("dim,n", [(2, 4), (2, 6), (3, 3)])
def test_coupling_blocks_match_the_upwind_face_integral(dim, n):
    """Every off-diagonal block of the assembled operator against the upwind
    face term written out from the weak form (Sec. 3.4.1, the face part of eq.
    jac-entries), integrated exactly on polynomials: for a trial function u on
    the neighbour f across face (axis, side) of element e and a test function v
    on e, v^T G_ef u = tau u_face int v(x_axis = side) u_f(x_axis = 1 - side)
    over the face when the face is an inflow face of e (u_face < 0), else 0.
    This fixes the sign, the face pairing (the neighbour's opposite face) and
    the neighbour table independently of the oracle's coupling code."""
    from tests.test_oracle_blocks import integral, poly_eval, restrict
    from scipy import signal
    mesh = 3
    params, nbr = synth.mesh_params(mesh, dim, seed=40 + n)
    G = operator.assemble(params, nbr, n, dim).toarray()
    T = tables(n)
    N = n ** dim
    rng = np.random.default_rng(n)
    checked = inflow = 0
    for e in range(mesh ** dim):
        for ax in range(dim):
            for side in (0, 1):
                f = int(nbr[e, 2 * ax + side])
                B = G[e * N:(e + 1) * N, f * N:(f + 1) * N]
                cu = rng.standard_normal((n,) * dim)
                cv = rng.standard_normal((n,) * dim)
                u = poly_eval(cu, T["x"])
                v = poly_eval(cv, T["x"])
                uf = params[e, 8 + 2 * ax + side]
                want = 0.0
                if uf < 0.0:
                    face = signal.convolve(restrict(cv, ax, float(side)), restrict(cu, ax, float(1 - side)))
                    want = params[e, 6] * uf * (integral(face) if dim > 1 else face)
                    inflow += 1
                got = v @ B @ u
                assert abs(got - want) <= 1e-12 * (1.0 + abs(want)) * n, (e, ax, side, got, want)
                checked += 1
    assert checked == (mesh ** dim) * 2 * dim and 0 < inflow < checked


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
