"""Pins of the oracle's element blocks against the weak form integrated exactly.

With alpha = 0 every term of the block is an integral of a polynomial that the
n-point Gauss rule integrates exactly (degree <= 2p in each variable), so
v^T A u must equal the weak form (mass, tau*beta*int u dv/dx_k, tau*nu*int grad u.grad v,
upwind outflow face terms; Sec. 3.4 and eq. weak-form) evaluated in exact
polynomial arithmetic on monomial coefficients.  This fixes the Kronecker
order (x slowest), the S = D^T W orientation and the face-term convention.
"""
import itertools

import numpy as np
import pytest
from scipy import integrate, signal

from oracle.blocks import element_block
from oracle.tables import tables


def poly_eval(c, pts):
    """c[a,b,(c)] monomial coefficients evaluated at tensor points, nodal order."""
    d = c.ndim
    grids = np.meshgrid(*([pts] * d), indexing="ij")
    out = np.zeros_like(grids[0])
    for idx in itertools.product(*[range(s) for s in c.shape]):
        term = c[idx]
        for g, k in zip(grids, idx):
            term = term * g ** k
        out = out + term
    return out.ravel()


def integral(c):
    out = 0.0
    for idx in itertools.product(*[range(s) for s in c.shape]):
        out += c[idx] / np.prod([k + 1 for k in idx])
    return out


def deriv(c, ax):
    k = np.arange(c.shape[ax]).reshape([-1 if i == ax else 1 for i in range(c.ndim)])
    return np.delete(c * k, 0, axis=ax)


def restrict(c, ax, t):
    """u restricted to the face x_ax = t (one variable fewer)."""
    k = np.arange(c.shape[ax]).reshape([-1 if i == ax else 1 for i in range(c.ndim)])
    return (c * t ** k).sum(axis=ax)


def weak_form(cu, cv, rec, dim):
    tau = rec[6]
    val = integral(signal.convolve(cu, cv))
    for ax in range(dim):
        val += tau * rec[ax] * integral(signal.convolve(cu, deriv(cv, ax)))
        val += tau * rec[3] * integral(signal.convolve(deriv(cu, ax), deriv(cv, ax)))
        for side in (0, 1):
            u = rec[8 + 2 * ax + side]
            if rec[7] != 0.0 and u > 0.0:
                t = float(side)
                val += tau * u * integral(signal.convolve(restrict(cu, ax, t), restrict(cv, ax, t)))
    return val


@pytest.mark.parametrize("dim,n,face", [(2, 3, 0), (2, 5, 1), (2, 8, 1), (3, 3, 1), (3, 4, 0)])
def test_bilinear_form_matches_weak_form(dim, n, face):
    rng = np.random.default_rng(7 + n)
    T = tables(n)
    for trial in range(3):
        rec = np.zeros(16)
        rec[:dim] = rng.uniform(-1, 1, dim)
        rec[3] = 10 ** rng.uniform(-3, -1)
        rec[4] = 0.0
        rec[6] = 0.1
        rec[7] = face
        rec[8:8 + 2 * dim] = rng.uniform(-1, 1, 2 * dim)  # face normal velocities
        A = element_block(rec, n, dim, T)
        cu = rng.standard_normal((n,) * dim)
        cv = rng.standard_normal((n,) * dim)
        u = poly_eval(cu, T["x"])
        v = poly_eval(cv, T["x"])
        exact = weak_form(cu, cv, rec, dim)
        assert abs(v @ A @ u - exact) < 1e-11 * (1 + abs(exact)) * n


def test_mass_coefficient_integral():
    # with tau = 0 the block is the mass term alone; its entries sum to the
    # n-point rule of int (1 + alpha sin(pi x y + phi)), spectrally accurate
    n = 16
    T = tables(n)
    rec = np.zeros(16)
    rec[4], rec[5], rec[6] = 0.37, 1.3, 0.0
    A = element_block(rec, n, 2, T)
    assert np.count_nonzero(A - np.diag(A.diagonal())) == 0
    ref, _ = integrate.dblquad(lambda y, x: 1 + 0.37 * np.sin(np.pi * x * y + 1.3), 0, 1, 0, 1,
                               epsabs=1e-14, epsrel=1e-14)
    assert abs(A.sum() - ref) < 1e-12


def test_alpha_zero_is_separable():
    n = 6
    T = tables(n)
    rec = np.array([0.3, -0.7, 0, 0.02, 0.0, 0.4, 0.1, 1, 0.3, -0.3, -0.7, 0.7, 0, 0, 0, 0])
    A = element_block(rec, n, 2, T)
    W = T["W"]
    X = W + 0.1 * (0.3 * T["S"] + 0.02 * T["K"]) + 0.1 * 0.3 * np.outer(T["l0"], T["l0"])
    Y = 0.1 * (-0.7 * T["S"] + 0.02 * T["K"]) + 0.1 * 0.7 * np.outer(T["l1"], T["l1"])
    np.testing.assert_allclose(A, np.kron(X, W) + np.kron(W, Y), atol=1e-13)
