"""Pins of the oracle's rearrangement and KSVD (Sec. 4.1, Sec. 4.3.1)."""
import numpy as np
import pytest

import synth
from oracle.blocks import element_block
from oracle.ksvd import canonical_sign, ksvd, ksvd2d, ksvd3d, precond_matrix, rearrange
from oracle.tables import tables


def test_rearrange_index_formula_by_loops():
    rng = np.random.default_rng(0)
    m1, n1, m2, n2 = 2, 3, 4, 2
    A = rng.standard_normal((m1 * m2, n1 * n2))
    R = rearrange(A, m1, n1, m2, n2)
    for i in range(m1):
        for j in range(n1):
            for k in range(m2):
                for l in range(n2):
                    assert R[i * n1 + j, k * n2 + l] == A[i * m2 + k, j * n2 + l]
    assert abs(np.linalg.norm(R) - np.linalg.norm(A)) < 1e-13


def test_rearrange_of_kron_is_rank_one():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((3, 4))
    Y = rng.standard_normal((2, 5))
    R = rearrange(np.kron(X, Y), 3, 4, 2, 5)
    np.testing.assert_allclose(R, np.outer(X.ravel(), Y.ravel()), atol=1e-14)


def test_rank_one_recovery():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((5, 5))
    Y = rng.standard_normal((5, 5))
    s, As, Bs = ksvd(np.kron(X, Y), 5, 5, 5, 5, 1)
    assert abs(s[0] - np.linalg.norm(X) * np.linalg.norm(Y)) < 1e-12 * s[0]
    assert s[1] < 1e-13 * s[0]
    np.testing.assert_allclose(np.kron(As[0], Bs[0]), np.kron(X, Y), atol=1e-12 * s[0])


@pytest.mark.parametrize("n,dim", [(4, 2), (8, 2), (16, 2), (4, 3)])
def test_eckart_young_residual(n, dim):
    params = synth.draw_params(6, dim, seed=11, face=True)
    T = tables(n)
    for rec in params:
        A = element_block(rec, n, dim, T)
        if dim == 2:
            for r in (1, 2, 3):
                s, As, Bs = ksvd(A, n, n, n, n, r)
                P = sum(np.kron(a, b) for a, b in zip(As, Bs))
                res2 = np.linalg.norm(A - P) ** 2
                assert abs(res2 - np.sum(s[r:] ** 2)) < 1e-13 * np.sum(s ** 2)
        else:
            s, As, Bs = ksvd(A, n, n, n * n, n * n, 1)
            res2 = np.linalg.norm(A - np.kron(As[0], Bs[0])) ** 2
            assert abs(res2 - np.sum(s[1:] ** 2)) < 1e-13 * np.sum(s ** 2)


def test_alpha_zero_2d_block_is_exact_rank_two():
    # Sec. 5.1: a separable operator is reproduced exactly by A1(x)B1 + A2(x)B2
    n = 8
    rec = np.array([0.4, -0.9, 0, 0.01, 0.0, 0, 0.1, 1, 0.4, -0.4, -0.9, 0.9, 0, 0, 0, 0])
    A = element_block(rec, n, 2)
    f = ksvd2d(A, n, 2)
    assert f["sigma"][2] < 1e-14 * f["sigma"][0]
    np.testing.assert_allclose(precond_matrix(f), A, atol=1e-13 * np.abs(A).max())


def test_separable_3d_block_is_exact():
    # beta_x = nu = alpha = 0: A = W (x) (W(x)W + tau*beta_y S(x)W + tau*beta_z W(x)S)
    n = 5
    rec = np.array([0.0, 0.6, -0.3, 0.0, 0.0, 0, 0.1, 0, 0, 0, 0, 0, 0, 0, 0, 0])
    A = element_block(rec, n, 3)
    f = ksvd3d(A, n)
    assert f["sigma1"][1] < 1e-14 * f["sigma1"][0]
    assert f["sigma2"][2] < 1e-14 * f["sigma2"][0]
    np.testing.assert_allclose(precond_matrix(f), A, atol=1e-13 * np.abs(A).max())


def test_canonical_sign():
    assert canonical_sign(np.array([0.1, -0.5, 0.5])) == -1.0
    assert canonical_sign(np.array([0.1, 0.5, -0.5])) == 1.0
    n = 6
    A = element_block(synth.draw_params(1, 2, seed=3)[0], n, 2)
    f = ksvd2d(A, n, 2)
    for a in f["A"]:
        k = np.argmax(np.abs(a.ravel()))
        assert a.ravel()[k] > 0
