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
        ok, _, _ = mlp.accept(A, F, dim, n)
        assert ok


def test_adam_step_closed_form():
    # first step: m^ = g, v^ = g^2, so the update is lr * g / (|g| + eps)
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    q, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(q, p - 0.01 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
