"""Pins of the oracle's systems blocks (oracle/systems.py), CPU only."""
import numpy as np

import synth
from oracle import systems
from oracle.apply import dense_solve
from oracle.blocks import element_block
from oracle.ksvd import precond_matrix, rearrange


def test_one_component_is_the_scalar_block():
    n = 5
    sd = synth.systems_elements(3, 1, seed=3)
    for e in range(3):
        A = systems.element_block(sd, e, n)
        rec = np.zeros(16)
        rec[0], rec[1] = -sd["J"][e, 0, 0, 0], -sd["J"][e, 1, 0, 0]
        rec[3], rec[4], rec[5], rec[6], rec[7] = sd["nu"][e], sd["alpha"][e], sd["phi"][e], sd["tau"], 1.0
        # outflow normal velocities: low face (-J)^+, high face (J)^+ (scalar: u_f = max(a.n, 0))
        rec[8], rec[9] = sd["Jm"][e, 0, 0, 0], sd["Jp"][e, 0, 0, 0]
        rec[10], rec[11] = sd["Jm"][e, 1, 0, 0], sd["Jp"][e, 1, 0, 0]
        np.testing.assert_allclose(A, element_block(rec, n, 2), atol=1e-14 * np.abs(A).max())


def test_separable_system_is_exact_rank_two():
    """alpha = nu = 0, no faces: A = (I (x) W + tau(-J_x) (x) S) (x) W + (-tau J_y (x) W) (x) S,
    two Kronecker terms with nc n x nc n first factors: the KSVD reproduces A."""
    n, nc = 6, 3
    sd = synth.systems_elements(2, nc, seed=4, face=False)
    sd["alpha"][:] = 0.0
    sd["nu"][:] = 0.0
    A = systems.element_block(sd, 1, n)
    f = systems.ksvd_system(A, nc, n, 2)
    assert f["sigma"][2] < 1e-14 * f["sigma"][0]
    np.testing.assert_allclose(precond_matrix(f), A, atol=1e-13 * np.abs(A).max())
    # the first factors act on (component, x): by loops on one entry
    R = rearrange(A, nc * n, nc * n, n, n)
    i, j, k, l = 7, 11, 2, 4
    assert R[i * nc * n + j, k * n + l] == A[i * n + k, j * n + l]


def test_eckart_young_and_dense_solve():
    n, nc = 5, 4
    sd = synth.systems_elements(2, nc, seed=5)
    for e in range(2):
        A = systems.element_block(sd, e, n)
        f = systems.ksvd_system(A, nc, n, 2)
        P = precond_matrix(f)
        res2 = np.linalg.norm(A - P) ** 2
        assert abs(res2 - np.sum(f["sigma"][2:] ** 2)) < 1e-12 * np.sum(f["sigma"] ** 2)
        r = np.random.default_rng(e).standard_normal(nc * n * n)
        z = dense_solve(f, r)
        assert np.linalg.norm(P @ z - r) <= 1e-10 * np.linalg.norm(r)
        blocks = systems.small_blocks(A, nc, n)
        assert len(blocks) == nc and blocks[0].shape == (n * n, n * n)
        np.testing.assert_array_equal(blocks[2], A[2 * n * n:3 * n * n, 2 * n * n:3 * n * n])
