"""Pins of the oracle's learned-setup pieces (oracle/mlp.py), CPU only."""
import numpy as np
import pytest

import synth
from oracle import mlp
from oracle.blocks import coefficient, element_block
from oracle.ksvd import factor_array, factors_from_array, ksvd2d, ksvd3d, precond_matrix


def rand_params(I, H, O, seed):
    rng = np.random.default_rng(seed)
    sizes = [H * I, H, H * H, H, O * H, O]
    return rng.standard_normal(sum(sizes)) * 0.3


@pytest.mark.parametrize("dim", [2, 3])
def test_features_match_the_coefficient_definition(dim):
    rec = synth.draw_params(5, dim, 17)
    F = mlp.features(rec, dim)
    assert F.shape == (5, 12)
    for e in range(5):
        assert F[e, 3] == pytest.approx(np.log10(rec[e, 3]))
        assert F[e, 6] ** 2 + F[e, 7] ** 2 == pytest.approx(1.0)
        # c at the reference points through the block generator's own coefficient
        for q, pt in enumerate(mlp.REF_POINTS):
            x = pt[:dim]
            if dim == 2:
                c = 1.0 + rec[e, 4] * np.sin(np.pi * x[0] * x[1] + rec[e, 5])
            else:
                c = 1.0 + rec[e, 4] * np.sin(np.pi * x[0] * x[1] * x[2] + rec[e, 5])
            assert F[e, 8 + q] == pytest.approx(c, rel=1e-15)
        # at the nodes of n = 1 (x = 1/2) the generator gives the same formula
        assert coefficient(rec[e], np.array([0.5]), dim)[0] == pytest.approx(
            1.0 + rec[e, 4] * np.sin(np.pi * 0.5 ** dim + rec[e, 5]))


@pytest.mark.parametrize("dim,n", [(2, 3), (3, 2)])
def test_gradient_by_central_differences(dim, n):
    I, H = 12, 7
    O = mlp.n_outputs(dim, n)
    p = rand_params(I, H, O, 1)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((5, I))
    t = rng.standard_normal((5, O))
    loss, g = mlp.loss_and_grad(p, x, t, I, H, O, dim, n)
    # the sign choice must be stable under the perturbation for the check to hold
    y, _ = mlp.forward(p, x, I, H, O)
    _, _, _, costs = mlp.loss_and_grad_y(y, t, dim, n)
    srt = np.sort(costs, axis=1)
    assert np.all(srt[:, 1] - srt[:, 0] > 1e-3)
    h = 1e-6
    idx = rng.choice(p.size, 60, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = mlp.loss_and_grad(p + e, x, t, I, H, O, dim, n)
        lm, _ = mlp.loss_and_grad(p - e, x, t, I, H, O, dim, n)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i]), np.max(np.abs(g)) * 1e-3), i


@pytest.mark.parametrize("dim,n", [(2, 4), (3, 3)])
def test_sign_patterns_leave_P_unchanged_and_loss_invariant(dim, n):
    rec = synth.draw_params(1, dim, 23, face=(dim == 3))[0]
    A = element_block(rec, n, dim)
    f = ksvd3d(A, n) if dim == 3 else ksvd2d(A, n, 2)
    F = factor_array(f)
    P = precond_matrix(f)
    for s in mlp.sign_patterns(dim):
        Fs = F * s[:, None, None]
        assert np.max(np.abs(precond_matrix(factors_from_array(Fs, dim)) - P)) <= 1e-14 * np.max(np.abs(P))
    O = F.size
    y = np.random.default_rng(3).standard_normal((1, O))
    base, _, _, _ = mlp.loss_and_grad_y(y, F.reshape(1, -1), dim, n)
    for s in mlp.sign_patterns(dim):
        ls, _, _, _ = mlp.loss_and_grad_y(y, (F * s[:, None, None]).reshape(1, -1), dim, n)
        assert ls == pytest.approx(base, rel=1e-14)
        # the exact target, in any of its sign forms, has zero loss
        z, _, _, _ = mlp.loss_and_grad_y((F * s[:, None, None]).reshape(1, -1), F.reshape(1, -1), dim, n)
        assert z == 0.0


@pytest.mark.parametrize("dim,n", [(2, 6), (3, 4)])
def test_residual_and_proxy_identities(dim, n):
    rec = synth.draw_params(3, dim, 29, face=(dim == 3))
    for r in rec:
        A = element_block(r, n, dim)
        f = ksvd3d(A, n) if dim == 3 else ksvd2d(A, n, 2)
        F = factor_array(f)
        res = mlp.residual(A, F, dim)
        prox = mlp.proxy_residual(A, F, dim, n)
        # the SVD's own subspaces: the proxy is the SVD residual
        assert prox == pytest.approx(res, rel=1e-9, abs=1e-14 * np.sum(A * A))
        if dim == 2:
            # Eckart-Young: the residual is the energy of the discarded singular values
            from oracle.ksvd import rearrange
            s = np.linalg.svd(rearrange(A, n, n, n, n), compute_uv=False)
            assert res == pytest.approx(np.sum(s[2:] ** 2), rel=1e-9, abs=1e-14 * s[0] ** 2)
        # a perturbed prediction: the proxy completes its left subspaces
        # optimally, so it never exceeds the prediction's own residual
        Fp = F + 0.05 * np.random.default_rng(5).standard_normal(F.shape) * np.abs(F).max()
        assert mlp.residual(A, Fp, dim) >= mlp.proxy_residual(A, Fp, dim, n) - 1e-12 * np.sum(A * A)


def test_adam_step_closed_form():
    # first step: m^ = g, v^ = g^2, so the update is lr * g / (|g| + eps)
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    q, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(q, p - 0.01 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def orth_pair(rng, n):
    """Two n x n matrices, orthogonal in the Frobenius inner product."""
    X = rng.standard_normal((n, n)) + 3 * np.eye(n)
    Y = rng.standard_normal((n, n))
    Y -= np.sum(X * Y) / np.sum(X * X) * X
    return X, Y


def constructed_case(dim, n, seed, noise=0.3, cond=1e-2):
    """A block with a known KSVD: A = P0 + N, whose rearrangement N is
    orthogonal to P0's singular vectors on both sides, so the SVD's factors are
    P0's; the first factor has a smallest singular value cond times its largest."""
    from oracle.ksvd import rearrange
    rng = np.random.default_rng(seed)
    Uq, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Vq, _ = np.linalg.qr(rng.standard_normal((n, n)))
    X1 = Uq @ np.diag(np.linspace(1.0, cond, n)) @ Vq
    if dim == 2:
        _, X2 = orth_pair(rng, n)
        X2 -= np.sum(X1 * X2) / np.sum(X1 * X1) * X1
        Y1, Y2 = orth_pair(rng, n)
        P0 = np.kron(X1, Y1) + 0.3 * np.kron(X2, Y2)
        shape = (n, n, n, n)
        L = np.stack([X1.ravel(), X2.ravel()], 1)
        R = np.stack([Y1.ravel(), Y2.ravel()], 1)
    else:
        Y1, Y2 = orth_pair(rng, n)
        Z1, Z2 = orth_pair(rng, n)
        D = np.kron(Y1, Z1) + 0.3 * np.kron(Y2, Z2)
        P0 = np.kron(X1, D)
        shape = (n, n, n * n, n * n)
        L = X1.ravel()[:, None]
        R = D.ravel()[:, None]
    R0 = rearrange(P0, *shape)
    G = rng.standard_normal(R0.shape)
    Ql, _ = np.linalg.qr(L)
    Qr, _ = np.linalg.qr(R)
    G = G - Ql @ (Ql.T @ G)
    G = G - (G @ Qr) @ Qr.T
    G *= noise * np.linalg.norm(R0) / np.linalg.norm(G)
    # back from the rearranged layout (the rearrangement is a permutation)
    N = np.zeros_like(P0)
    idx = np.arange(P0.size).reshape(P0.shape)
    perm = rearrange(idx, *shape).ravel()
    N.ravel()[perm] = G.ravel()
    A = P0 + N
    f = ksvd3d(A, n) if dim == 3 else ksvd2d(A, n, 2)
    return A, factor_array(f), f


@pytest.mark.parametrize("dim,n", [(2, 5), (3, 4)])
def test_accept_branches(dim, n):
    from oracle.apply import dense_solve
    A, F, f = constructed_case(dim, n, 41)
    # the SVD reproduces the construction: the first factor is ill-conditioned
    s0 = np.linalg.svd(F[0], compute_uv=False)
    assert s0[-1] / s0[0] == pytest.approx(1e-2, rel=1e-6)
    # the SVD's own factors: equal residuals, E = 0
    ok, rp, rs, g = mlp.accept(A, F, F, dim)
    assert ok and rp == pytest.approx(rs, rel=1e-12) and g <= 1e-12
    assert rs == pytest.approx(0.3 * np.linalg.norm(A - 0.0 * A) / np.sqrt(1.09), rel=0.2)
    # a mild perturbation is taken
    Fm = F * (1.0 + 1e-7 * np.random.default_rng(2).standard_normal(F.shape))
    ok, rp, rs, g = mlp.accept(A, Fm, F, dim)
    assert ok and rp <= 1.1 * rs and g <= 0.01
    # a larger one passes the looser guard 0.1; the guard grows with the
    # perturbation (the first factor's condition number is 100)
    Fm5 = F * (1.0 + 1e-5 * np.random.default_rng(2).standard_normal(F.shape))
    ok5, _, _, g5 = mlp.accept(A, Fm5, F, dim, guard=0.1)
    assert ok5 and g5 > 10 * g
    # rescaled prediction: the residual grows past 1.1 x the SVD's
    Fs = F.copy()
    Fs[0] *= 0.5
    ok, rp, rs, g = mlp.accept(A, Fs, F, dim)
    assert not ok and rp > 1.1 * rs
    # all-zero prediction: explains nothing
    ok, rp, rs, g = mlp.accept(A, np.zeros_like(F), F, dim)
    assert not ok and rp == pytest.approx(np.linalg.norm(A), rel=1e-14)
    # near-singular prediction: remove (1 - 1e-6) of the smallest singular
    # direction of the first factor.  The Frobenius change is 1% of ||A||,
    # far inside the 1.1 x bar, but P_pred is nearly singular: the guard
    # rejects it
    U, s, Vt = np.linalg.svd(F[0])
    Fn = F.copy()
    Fn[0] = F[0] - (1.0 - 1e-6) * s[-1] * np.outer(U[:, -1], Vt[-1])
    ok, rp, rs, g = mlp.accept(A, Fn, F, dim)
    assert rp <= 1.1 * rs, (rp, rs)
    assert not ok and g > 0.1
    # the estimate is a lower bound of the exact norm, and of its order here
    Pp = precond_matrix(factors_from_array(Fn, dim))
    E = np.stack([dense_solve(f, Pp[:, k]) for k in range(Pp.shape[0])], axis=1) - np.eye(Pp.shape[0])
    exact = np.linalg.norm(E, 2)
    assert g <= exact * (1 + 1e-9) and g >= 0.2 * exact
