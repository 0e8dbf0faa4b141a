"""Learned setup: a small MLP from element features to Kronecker factors.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper forms the factors by an SVD of the rearranged block (Sec. 4.1).
The learned variant predicts them from the element's record and keeps the SVD
as the arbiter.  Everything here is the plain FP64 definition:

features(rec, dim): 12 numbers per element
    beta_x, beta_y, beta_z (0 in 2D), log10 nu, tau, alpha, sin phi, cos phi,
    and the mass coefficient c = 1 + alpha sin(pi x y [z] + phi) at the
    reference points (1/4,1/4,1/4), (3/4,1/4,3/4), (1/4,3/4,3/4), (3/4,3/4,1/4)
    (2D: the same (x, y), no z).

Network (row-major weights, the layout of the GPU model buffer):
    h1 = silu(W1 xn + b1), h2 = silu(W2 h1 + b2), y = W3 h2 + b3,
    W1: H x 12, W2: H x H, W3: O x H; silu(z) = z / (1 + exp(-z));
    xn = (x - x_mean) / x_std; the outputs are the factors divided by a
    per-block scale (no shift, so sign changes commute with the scaling).

Outputs: the canonical factor stack (``ksvd.factor_array``): 3D
[A1, B1, C1, B2, C2], 2D rank 2 [A1, B1, A2, B2], each n x n row-major.

Loss: the factors are defined up to sign changes that leave P unchanged
(3D: A1 -> s0 A1, B_j -> s_j B_j, C_j -> s0 s_j C_j; 2D: (A_j, B_j) -> s_j
(A_j, B_j)).  Per sample the target is taken with the sign pattern closest
to the prediction:  L = 1/(N O) sum_samples min_s ||y - s . t||^2.

Residuals: res(A, f) = ||A - P(f)||_F^2 by dense assembly; the Rayleigh-Ritz
proxy of a prediction keeps only its left subspaces and completes them
optimally (2D: U = orth[vec A1, vec A2], proxy = ||A||^2 - ||U^T R(A)||_F^2;
3D: u = vec A1 / ||vec A1||, D = unvec(R(A)^T u), U2 = orth[vec B1, vec B2],
proxy = ||A||^2 - ||U2^T R(D)||_F^2); it is never below the SVD's residual.

Acceptance (``accept``): the SVD's factors judge.  A prediction is used
directly when ||A - P_pred||_F <= 1.1 ||A - P_svd||_F (the rearranged
residual within 1.1 times the SVD's), ||A - P_pred||_F < ||A||_F, and the
spectral guard ||P_svd^{-1} P_pred - I||_2 <= 0.01 holds by a three-step power
estimate (``guard_estimate``).  The guard's default is the largest that keeps
FGMRES(30) on the 3D p = 15 workload within one iteration of the SVD's
factors (0.1 admits predictions that cost 32 more iterations).

Pinned by tests/test_oracle_mlp.py (central differences, sign invariance of
P and of the loss, residual identities, proxy = SVD residual on the SVD's
own subspaces, each acceptance branch on constructed predictions: the SVD's
own factors, a rescaled prediction, an all-zero prediction, and a
near-singular perturbation that keeps the Frobenius residual but fails the
guard, whose estimate is checked against the exact norm).
"""
from __future__ import annotations

import numpy as np

from .ksvd import factors_from_array, precond_matrix, rearrange

REF_POINTS = np.array([[0.25, 0.25, 0.25], [0.75, 0.25, 0.75], [0.25, 0.75, 0.75],
                       [0.75, 0.75, 0.25]])
N_FEATURES = 12


def features(rec: np.ndarray, dim: int) -> np.ndarray:
    rec = np.atleast_2d(rec)
    out = np.zeros((rec.shape[0], N_FEATURES))
    out[:, 0] = rec[:, 0]
    out[:, 1] = rec[:, 1]
    out[:, 2] = rec[:, 2] if dim == 3 else 0.0
    out[:, 3] = np.log10(rec[:, 3])
    out[:, 4] = rec[:, 6]
    out[:, 5] = rec[:, 4]
    out[:, 6] = np.sin(rec[:, 5])
    out[:, 7] = np.cos(rec[:, 5])
    for q, (x, y, z) in enumerate(REF_POINTS):
        prod = x * y * z if dim == 3 else x * y
        out[:, 8 + q] = 1.0 + rec[:, 4] * np.sin(np.pi * prod + rec[:, 5])
    return out


def sign_patterns(dim: int) -> np.ndarray:
    """Rows: the sign of each factor block under every P-preserving change."""
    rows = []
    if dim == 3:
        for s0 in (1, -1):
            for s1 in (1, -1):
                for s2 in (1, -1):
                    rows.append([s0, s1, s0 * s1, s2, s0 * s2])
    else:
        for s1 in (1, -1):
            for s2 in (1, -1):
                rows.append([s1, s1, s2, s2])
    return np.array(rows, dtype=np.float64)


def n_outputs(dim: int, n: int) -> int:
    return (5 if dim == 3 else 4) * n * n


def unpack(params: np.ndarray, I: int, H: int, O: int):
    p = np.asarray(params, dtype=np.float64)
    sizes = [H * I, H, H * H, H, O * H, O]
    assert p.size == sum(sizes)
    parts = np.split(p, np.cumsum(sizes)[:-1])
    return (parts[0].reshape(H, I), parts[1], parts[2].reshape(H, H), parts[3],
            parts[4].reshape(O, H), parts[5])


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, xn: np.ndarray, I: int, H: int, O: int):
    """Outputs (N x O) and the pre-activations for the backward pass."""
    W1, b1, W2, b2, W3, b3 = unpack(params, I, H, O)
    z1 = xn @ W1.T + b1
    h1 = silu(z1)
    z2 = h1 @ W2.T + b2
    h2 = silu(z2)
    y = h2 @ W3.T + b3
    return y, (xn, z1, h1, z2, h2)


def block_signs(dim: int, n: int) -> np.ndarray:
    """patterns (P x O): the sign of every output under every pattern."""
    pat = sign_patterns(dim)
    return np.repeat(pat, n * n, axis=1)


def loss_and_grad_y(y: np.ndarray, t: np.ndarray, dim: int, n: int):
    """Sign-minimised MSE and its gradient with respect to y."""
    S = block_signs(dim, n)                         # P x O
    N, O = y.shape
    # per sample and pattern: sum_o (y - s t)^2
    costs = np.stack([np.sum((y - s * t) ** 2, axis=1) for s in S], axis=1)  # N x P
    best = np.argmin(costs, axis=1)
    st = S[best] * t
    loss = float(np.sum(costs[np.arange(N), best]) / (N * O))
    gy = 2.0 * (y - st) / (N * O)
    return loss, gy, best, costs


def loss_and_grad(params, xn, t, I, H, O, dim, n):
    """Loss and the gradient with respect to the flat parameter vector."""
    W1, b1, W2, b2, W3, b3 = unpack(params, I, H, O)
    y, (x, z1, h1, z2, h2) = forward(params, xn, I, H, O)
    loss, gy, _, _ = loss_and_grad_y(y, t, dim, n)
    gW3 = gy.T @ h2
    gb3 = gy.sum(axis=0)
    gh2 = gy @ W3
    gz2 = gh2 * silu_grad(z2)
    gW2 = gz2.T @ h1
    gb2 = gz2.sum(axis=0)
    gh1 = gz2 @ W2
    gz1 = gh1 * silu_grad(z1)
    gW1 = gz1.T @ x
    gb1 = gz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), step counted from 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def residual(A: np.ndarray, farr: np.ndarray, dim: int) -> float:
    """||A - P||_F^2 for a factor stack, by dense assembly."""
    P = precond_matrix(factors_from_array(np.asarray(farr, dtype=np.float64), dim))
    return float(np.sum((A - P) ** 2))


def _orth(cols: np.ndarray) -> np.ndarray:
    q, _ = np.linalg.qr(cols)
    return q


def proxy_residual(A: np.ndarray, farr: np.ndarray, dim: int, n: int) -> float:
    """Rayleigh-Ritz residual of the prediction's left subspaces (>= the optimum)."""
    a2 = float(np.sum(A * A))
    if dim == 2:
        R = rearrange(A, n, n, n, n)
        U = _orth(np.stack([farr[0].ravel(), farr[2].ravel()], axis=1))
        return a2 - float(np.sum((U.T @ R) ** 2))
    R1 = rearrange(A, n, n, n * n, n * n)
    u = farr[0].ravel() / np.linalg.norm(farr[0])
    D = (R1.T @ u).reshape(n * n, n * n)
    R2 = rearrange(D, n, n, n, n)
    U2 = _orth(np.stack([farr[1].ravel(), farr[3].ravel()], axis=1))
    return a2 - float(np.sum((U2.T @ R2) ** 2))


GUARD_STEPS = 3


def guard_estimate(f_pred: dict, f_svd: dict, steps: int = GUARD_STEPS) -> float:
    """Power estimate of ||P_svd^{-1} P_pred - I||_2 from the normalised ones
    vector: gamma = max_k ||E v_k||, v_{k+1} = E v_k / ||E v_k||, k < steps
    (each ||E v_k|| is a lower bound of the norm)."""
    from .apply import dense_solve
    Pp = precond_matrix(f_pred)
    N = Pp.shape[0]
    v = np.ones(N) / np.sqrt(N)
    gamma = 0.0
    for _ in range(steps):
        e = dense_solve(f_svd, Pp @ v) - v
        ne = float(np.linalg.norm(e))
        gamma = max(gamma, ne)
        if not ne > 0.0:
            break
        v = e / ne
    return gamma


def accept(A: np.ndarray, farr: np.ndarray, svd_farr: np.ndarray, dim: int, factor: float = 1.1,
           guard: float = 0.01, steps: int = GUARD_STEPS):
    """Acceptance test of a predicted factor stack against the SVD's.

    The prediction is used directly only when its rearranged residual is
    within ``factor`` of the SVD's, ||A - P_pred||_F <= factor ||A - P_svd||_F,
    when it explains part of A (||A - P_pred||_F < ||A||_F: an all-zero
    prediction is never taken), and when the spectral guard holds: the power
    estimate of ||P_svd^{-1} P_pred - I||_2 (``guard_estimate``) is at most
    ``guard``.  A Frobenius residual does not bound the spectrum of P_pred; the
    guard does, since with ||E|| <= g < 1, P_pred^{-1} A = (I + E)^{-1}
    P_svd^{-1} A differs from the SVD's preconditioned operator by at most
    g / (1 - g) relatively.  Returns (accepted, res_pred, res_svd, gamma),
    residuals as Frobenius norms."""
    res_p = np.sqrt(residual(A, farr, dim))
    res_s = np.sqrt(residual(A, svd_farr, dim))
    a = float(np.linalg.norm(A))
    frob = res_p <= factor * res_s and res_p < a
    gamma = guard_estimate(factors_from_array(np.asarray(farr, np.float64), dim),
                           factors_from_array(np.asarray(svd_farr, np.float64), dim), steps)
    return bool(frob and gamma <= guard), res_p, res_s, gamma
