"""Pins of the oracle's rearrangement and KSVD (Sec. 4.1, Sec. 4.3.1)."""
import numpy as np
import pytest

import synth
from oracle.blocks import element_block
from oracle.ksvd import (AXIS_ORDERS, canonical_sign, ksvd, ksvd2d, ksvd3d, ksvd3d_axis, ksvd3d_best_axis,
                         permute_block, precond_matrix, rearrange)
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


def test_permute_block_by_loops():
    n = 3
    A = np.random.default_rng(5).standard_normal((n ** 3, n ** 3))
    for order in AXIS_ORDERS.values():
        B = permute_block(A, n, order)
        for I in range(n ** 3):
            i = (I // 9, (I // 3) % 3, I % 3)
            for J in range(0, n ** 3, 5):
                j = (J // 9, (J // 3) % 3, J % 3)
                # new index q holds old axis order[q]
                oi = [0, 0, 0]
                oj = [0, 0, 0]
                for q in range(3):
                    oi[order[q]] = i[q]
                    oj[order[q]] = j[q]
                assert B[I, J] == A[oi[0] * 9 + oi[1] * 3 + oi[2], oj[0] * 9 + oj[1] * 3 + oj[2]]


@pytest.mark.parametrize("axis", [1, 2])
def test_split_axis_recovers_a_block_separable_along_that_axis(axis):
    """A = sum over the two other axes' terms with a single factor on `axis`:
    X (x) (Y1 (x) Z1 + Y2 (x) Z2) placed so that X acts on `axis`.  The KSVD
    split on `axis` reproduces A exactly; the paper's fixed split of the
    first axis does not; the best-axis rule picks `axis`."""
    n = 4
    rng = np.random.default_rng(10 + axis)
    X, Y1, Z1, Y2, Z2 = (rng.standard_normal((n, n)) for _ in range(5))
    B = np.kron(X, np.kron(Y1, Z1) + np.kron(Y2, Z2))     # X on the first axis
    order = AXIS_ORDERS[axis]
    inv = [0, 0, 0]
    for q, o in enumerate(order):
        inv[o] = q
    A = permute_block(B, n, tuple(inv))                    # X on `axis`
    # by loops: A's entry with X's indices on `axis`
    i, j = (1, 2, 3), (3, 0, 2)
    other = [q for q in range(3) if q != axis]
    val = X[i[axis], j[axis]] * (Y1[i[other[0]], j[other[0]]] * Z1[i[other[1]], j[other[1]]] +
                                 Y2[i[other[0]], j[other[0]]] * Z2[i[other[1]], j[other[1]]])
    assert abs(A[i[0] * 16 + i[1] * 4 + i[2], j[0] * 16 + j[1] * 4 + j[2]] - val) < 1e-12
    f = ksvd3d_axis(A, n, axis)
    np.testing.assert_allclose(precond_matrix(f), A, atol=1e-12 * np.abs(A).max())
    f0 = ksvd3d(A, n)
    assert np.linalg.norm(A - precond_matrix(f0)) > 1e-3 * np.linalg.norm(A)
    best = ksvd3d_best_axis(A, n)
    assert best["axis"] == axis


def test_split_axis_zero_is_the_paper_split():
    n = 4
    A = element_block(synth.draw_params(1, 3, seed=8, face=True)[0], n, 3)
    f = ksvd3d_axis(A, n, 0)
    g = ksvd3d(A, n)
    np.testing.assert_allclose(precond_matrix(f), precond_matrix(g), atol=1e-13 * np.abs(A).max())
