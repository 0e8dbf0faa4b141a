"""Pins of the oracle's 1D tables against closed forms and identities (Sec. 3.1-3.2)."""
import numpy as np
import pytest

from oracle.tables import gauss_legendre01, lagrange_values, tables

NS = [2, 3, 4, 8, 16, 31]


def test_closed_form_rules():
    # textbook two- and three-point Gauss-Legendre rules, mapped to [0,1]
    x, w = gauss_legendre01(2)
    np.testing.assert_allclose(x, [0.5 - 0.5 / np.sqrt(3), 0.5 + 0.5 / np.sqrt(3)], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, [0.5, 0.5], atol=1e-15)
    x, w = gauss_legendre01(3)
    np.testing.assert_allclose(x, [0.5 - 0.5 * np.sqrt(0.6), 0.5, 0.5 + 0.5 * np.sqrt(0.6)], atol=1e-15)
    np.testing.assert_allclose(w, [5 / 18, 8 / 18, 5 / 18], atol=1e-15)


@pytest.mark.parametrize("n", NS)
def test_quadrature_exactness(n):
    x, w = gauss_legendre01(n)
    for m in range(2 * n):
        assert abs(w @ x ** m - 1.0 / (m + 1)) < 1e-14 * max(1, n / 4)


@pytest.mark.parametrize("n", NS)
def test_derivative_of_monomials(n):
    T = tables(n)
    x = T["x"]
    for m in range(n):
        exact = m * x ** (m - 1) if m > 0 else 0 * x
        err = np.max(np.abs(T["D"] @ x ** m - exact))
        assert err < 1e-12 * n ** 2 * max(1.0, np.max(np.abs(exact)))


@pytest.mark.parametrize("n", NS)
def test_summation_by_parts_and_K(n):
    T = tables(n)
    S, K = T["S"], T["K"]
    sbp = S + S.T - (np.outer(T["l1"], T["l1"]) - np.outer(T["l0"], T["l0"]))
    assert np.max(np.abs(sbp)) < 1e-12 * n
    assert np.max(np.abs(K @ np.ones(n))) < 1e-11 * n ** 3
    assert np.max(np.abs(K - K.T)) < 1e-11 * n ** 3
    assert np.min(np.linalg.eigvalsh(0.5 * (K + K.T))) > -1e-9 * n ** 3


@pytest.mark.parametrize("n", NS)
def test_lagrange_boundary_values(n):
    T = tables(n)
    assert abs(T["l0"].sum() - 1.0) < 1e-12 and abs(T["l1"].sum() - 1.0) < 1e-12
    np.testing.assert_allclose(T["l0"][::-1], T["l1"], atol=1e-12)
    # phi_j is the Lagrange basis: interpolates x^m exactly for m <= p
    for m in range(n):
        assert abs(lagrange_values(T["x"], 1.0) @ T["x"] ** m - 1.0) < 1e-12 * n
        assert abs(lagrange_values(T["x"], 0.25) @ T["x"] ** m - 0.25 ** m) < 1e-12 * n
    # trace-inverse constant of the Gauss rule: l^T W^{-1} l = n^2
    assert abs(T["l1"] @ (T["l1"] / T["w"]) - n * n) < 1e-10 * n * n
