"""Pins of the oracle's preconditioner applies (Sec. 4.2-4.4, Algs. 5-8)."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle.apply import dense_solve, eig_fdm_solve, quasi_tri_sylvester, schur_solve
from oracle.blocks import element_block
from oracle.krylov import bj_factor, bj_solve
from oracle.ksvd import ksvd2d, ksvd3d, precond_matrix
from oracle.tables import tables

U = np.finfo(np.float64).eps


def factors(dim, n, count, seed, face=True):
    params = synth.draw_params(count, dim, seed=seed, face=face)
    T = tables(n)
    out = []
    for rec in params:
        A = element_block(rec, n, dim, T)
        out.append(ksvd2d(A, n, 2) if dim == 2 else ksvd3d(A, n))
    return out


@pytest.mark.parametrize("dim,n", [(2, 4), (2, 8), (2, 16), (3, 4), (3, 6)])
def test_dense_solve_residual(dim, n):
    rng = np.random.default_rng(n)
    for f in factors(dim, n, 3, 20 + n):
        P = precond_matrix(f)
        r = rng.standard_normal((2, n ** dim))
        z = dense_solve(f, r)
        for k in range(2):
            assert np.linalg.norm(P @ z[k] - r[k]) < 1e-12 * np.linalg.norm(P) * np.linalg.norm(z[k])


@pytest.mark.parametrize("dim,n", [(2, 4), (2, 8), (2, 16), (3, 4), (3, 8)])
def test_schur_route_equals_dense(dim, n):
    rng = np.random.default_rng(100 + n)
    for f in factors(dim, n, 4, 30 + n):
        r = rng.standard_normal(n ** dim)
        z = dense_solve(f, r)
        zs = schur_solve(f, r)
        kappa = np.linalg.cond(precond_matrix(f))
        assert np.linalg.norm(zs - z) / np.linalg.norm(z) < max(1e-12, 100 * kappa * U)


@pytest.mark.parametrize("n", [3, 4, 5, 6])
def test_fast_diagonalisation_equals_dense_small_n(n):
    rng = np.random.default_rng(200 + n)
    for f in factors(2, n, 5, 40 + n, face=False):
        r = rng.standard_normal(n * n)
        z = dense_solve(f, r)
        assert np.linalg.norm(eig_fdm_solve(f, r) - z) / np.linalg.norm(z) < 1e-12


def test_quasi_triangular_sylvester_against_scipy():
    rng = np.random.default_rng(5)
    for n in (3, 7, 12):
        T1, _ = sla.schur(rng.standard_normal((n, n)), output="real")
        T2, _ = sla.schur(rng.standard_normal((n, n)), output="real")
        assert np.any(np.abs(np.diag(T2, -1)) > 0)  # has 2x2 blocks
        F = rng.standard_normal((n, n))
        Y = quasi_tri_sylvester(T1, T2, F)
        Yref = sla.solve_sylvester(T1, T2.T, F)
        np.testing.assert_allclose(Y, Yref, rtol=1e-10, atol=1e-12)


def test_exact_case_ksvd_equals_block_jacobi():
    # Sec. 5.1: when the block is exactly rank 2 in Kronecker form, K and J coincide
    n = 8
    params = synth.draw_params(4, 2, seed=9, face=True)
    params[:, 4] = 0.0  # alpha = 0: separable
    T = tables(n)
    blocks = np.stack([element_block(rec, n, 2, T) for rec in params])
    r = np.random.default_rng(1).standard_normal((4, n * n))
    zj = bj_solve(bj_factor(blocks), r)
    for e in range(4):
        zk = schur_solve(ksvd2d(blocks[e], n, 2), r[e])
        assert np.linalg.norm(zk - zj[e]) / np.linalg.norm(zj[e]) < 1e-11
