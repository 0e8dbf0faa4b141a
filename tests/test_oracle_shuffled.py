"""Pins of the general-element oracle (oracle/shuffled.py): the block by its
quadrature definition and the sum-factorised shuffled products of Sec. 4.2.1
and Sec. 4.3.2, with their operation counts."""
import numpy as np
import pytest

import synth
from oracle import shuffled as sh
from oracle.apply import Flops
from oracle.blocks import coefficient, element_block
from oracle.tables import lagrange_derivative_matrix, tables


def record_as_general(rec, n, dim):
    """A structured record written as a general element at mu = n (collocation)."""
    T = tables(n)
    nd = n ** dim
    a = np.stack([np.full(nd, -rec[i]) for i in range(dim)])
    g = []
    for ax in range(dim):
        for side in (0, 1):
            u = rec[8 + 2 * ax + side] if rec[7] != 0.0 else 0.0
            g.append(np.full(n ** (dim - 1), max(u, 0.0)))
    return dict(dim=dim, n=n, mu=n, tau=rec[6], c=coefficient(rec, T["x"], dim), a=a,
                nu=np.full(nd, rec[3]), g=np.stack(g))


@pytest.mark.parametrize("dim,n", [(2, 3), (2, 6), (3, 3), (3, 4)])
def test_collocated_reduction_to_structured_block(dim, n):
    Q = sh.quad_tables(n, n)
    assert np.allclose(Q["Phi"], np.eye(n), atol=1e-13)
    assert np.allclose(Q["dPhi"], lagrange_derivative_matrix(Q["xn"]), rtol=1e-12, atol=1e-11)
    for rec in synth.draw_params(3, dim, 61 + n, face=True):
        A = sh.element_block(record_as_general(rec, n, dim), Q)
        Aref = element_block(rec, n, dim)
        assert np.max(np.abs(A - Aref)) <= 1e-12 * np.max(np.abs(Aref))


def poly_general(dim, n, mu, seed):
    """Fields that are polynomials of degree <= 2 per axis, evaluated at the
    mu-point rule: the block is then the same for every mu with 2 mu - 1 >= 2 (n - 1) + 2 + 2."""
    rng = np.random.default_rng(seed)
    cf = rng.standard_normal((dim + 2, 3, dim))          # per field, per axis, degree-2 coefficients
    xq = synth.quad_points01(mu)
    grid = [t.ravel() for t in np.meshgrid(*([xq] * dim), indexing="ij")]

    def field(k, X):
        out = 1.0
        for ax in range(dim):
            out = out * (cf[k, 0, ax] + cf[k, 1, ax] * X[ax] + cf[k, 2, ax] * X[ax] ** 2)
        return out
    c = 2.0 + field(0, grid) ** 2 * 0.0 + field(0, grid)
    a = np.stack([field(1 + i, grid) for i in range(dim)]) if dim == 2 else \
        np.stack([field(1 + i % (dim + 1), grid) for i in range(dim)])
    nu = field(dim + 1, grid)
    g = []
    for ax in range(dim):
        for side in (0, 1):
            rest = [t.ravel() for t in np.meshgrid(*([xq] * (dim - 1)), indexing="ij")]
            X = rest[:ax] + [np.full(mu ** (dim - 1), float(side))] + rest[ax:]
            g.append(field(ax + 1, X))
    return dict(dim=dim, n=n, mu=mu, tau=0.1, c=c, a=a, nu=nu, g=np.stack(g))


@pytest.mark.parametrize("dim,n", [(2, 4), (3, 3)])
def test_exact_integration_independent_of_mu(dim, n):
    # degree per axis of an integrand: 2 (n - 1) + 2; exact when 2 mu - 1 >= that
    mus = [n + 1, n + 3]
    blocks = [sh.element_block(poly_general(dim, n, mu, 7), sh.quad_tables(n, mu)) for mu in mus]
    assert np.max(np.abs(blocks[0] - blocks[1])) <= 1e-12 * np.max(np.abs(blocks[1]))


@pytest.mark.parametrize("dim,n,mu", [(2, 5, 7), (3, 3, 5)])
def test_mass_and_advection_closed_forms(dim, n, mu):
    Q = sh.quad_tables(n, mu)
    nd, md = n ** dim, mu ** dim
    zero = dict(dim=dim, n=n, mu=mu, tau=1.0, c=np.zeros(md), a=np.zeros((dim, md)), nu=np.zeros(md),
                g=np.zeros((2 * dim, mu ** (dim - 1))))
    mass = dict(zero, c=np.ones(md))
    M = sh.element_block(mass, Q)
    # the unit square's area, and int phi_I = the n-point Gauss weights (exact for degree n - 1)
    assert np.sum(M) == pytest.approx(1.0, rel=1e-13)
    w = tables(n)["w"]
    wd = w
    for _ in range(dim - 1):
        wd = np.multiply.outer(wd, w).ravel()
    assert np.allclose(M.sum(axis=1), wd, rtol=1e-12, atol=1e-15)
    # constant velocity: the test functions sum to 1, whose gradient vanishes
    adv = dict(zero, a=np.ones((dim, md)) * np.arange(1, dim + 1)[:, None])
    V = sh.element_block(adv, Q)
    assert np.max(np.abs(V.sum(axis=0))) <= 1e-12 * np.max(np.abs(V))


@pytest.mark.parametrize("dim,n,mu", [(2, 4, 4), (2, 5, 7), (3, 3, 3), (3, 4, 6)])
def test_shuffled_products_equal_explicit_rearrangement(dim, n, mu):
    q = synth.quad_elements(2, dim, mu, seed=90 + n)
    Q = sh.quad_tables(n, mu)
    rng = np.random.default_rng(n)
    for e in range(2):
        el = synth.quad_element(q, e, n)
        R = sh.explicit_rearranged(el, Q)
        v = rng.standard_normal(R.shape[1])
        u = rng.standard_normal(R.shape[0])
        Rv = sh.shuffled_matvec(el, Q, v)
        Rtu = sh.shuffled_rmatvec(el, Q, u)
        assert np.linalg.norm(Rv - R @ v) <= 1e-12 * np.linalg.norm(R) * np.linalg.norm(v)
        assert np.linalg.norm(Rtu - R.T @ u) <= 1e-12 * np.linalg.norm(R) * np.linalg.norm(u)


def slope(ns, counts):
    return float(np.polyfit(np.log(ns), np.log(counts), 1)[0])


def test_shuffled_product_operation_counts():
    """2D: O(p^3) per product (Sec. 4.2.1); 3D stage 1: O(p^5) (Sec. 4.3.2)."""
    out = {}
    for dim, ns, want in ((2, [4, 6, 8, 12, 16, 24, 31], 3.0), (3, [4, 6, 8, 11, 16, 22], 5.0)):
        counts = []
        for n in ns:
            mu = n + 1
            el = synth.quad_element(synth.quad_elements(1, dim, mu, seed=5), 0, n)
            Q = sh.quad_tables(n, mu)
            fc = Flops()
            sh.shuffled_matvec(el, Q, np.ones(n ** (2 * dim - 2)), fc)
            ft = Flops()
            sh.shuffled_rmatvec(el, Q, np.ones(n * n), ft)
            counts.append(fc.count + ft.count)
        # growth rate at the upper end of the range, where the lower-order
        # contractions (n^3 mu^2, n^2 mu^3, ...) no longer weigh in
        out[dim] = slope(ns[-3:], counts[-3:])
        assert abs(out[dim] - want) <= 0.25, (dim, out[dim], counts)
        assert slope(ns, counts) <= want + 0.1
    # the 3D first stage grows two powers of p faster than the 2D products
    assert out[3] - out[2] >= 1.7


def test_apply_operation_counts():
    """Algs. 6/8: about 14 n^3 (2D) and 16 n^4 (3D) operations per apply,
    O(p^{d+1}) (Sec. 4.4)."""
    from oracle.apply import SchurPrecond
    from oracle.ksvd import ksvd2d, ksvd3d
    for dim, ns, lead, want in ((2, [4, 6, 8, 12, 16, 24, 31], 14, 3.0), (3, [4, 6, 8, 12, 16], 16, 4.0)):
        counts = []
        for n in ns:
            rec = synth.draw_params(1, dim, 70 + n, face=True)[0]
            A = element_block(rec, n, dim)
            pc = SchurPrecond(ksvd3d(A, n) if dim == 3 else ksvd2d(A, n, 2))
            fc = Flops()
            pc.solve(np.random.default_rng(n).standard_normal(n ** dim), fc)
            counts.append(fc.count)
            # leading term, with the lower-order terms shrinking as 1/n
            assert abs(fc.count / (lead * n ** (dim + 1)) - 1.0) <= 1.0 / n, (dim, n, fc.count)
        assert abs(slope(ns, counts) - want) <= 0.15, (dim, counts)


def test_rearranged_rows_and_ksvd_from_them():
    """R(A) built row by row from the transpose products equals the explicit
    rearrangement, and the KSVD taken from it equals the one of the dense
    block (3D, n = 4, mu = 6)."""
    from oracle.ksvd import ksvd3d, ksvd3d_rearranged, precond_matrix
    n, mu = 4, 6
    q = synth.quad_elements(2, 3, mu, seed=31)
    Q = sh.quad_tables(n, mu)
    el = synth.quad_element(q, 1, n)
    R = sh.rearranged_rows(el, Q)
    np.testing.assert_allclose(R, sh.explicit_rearranged(el, Q), atol=1e-13 * np.abs(R).max())
    A = sh.element_block(el, Q)
    f1 = ksvd3d_rearranged(R, n)
    f2 = ksvd3d(A, n)
    np.testing.assert_allclose(f1["sigma2"][:3], f2["sigma2"][:3], rtol=1e-12)
    np.testing.assert_allclose(precond_matrix(f1), precond_matrix(f2), atol=1e-12 * np.abs(A).max())
