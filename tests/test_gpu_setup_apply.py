"""GPU parity of element source, setup and apply against the FP64 oracle.

Bars (stated per result):
  * explicit blocks: max |A_gpu - A_oracle| <= 1e-13 * max|A|;
  * singular values: relative <= 1e-12;
  * preconditioner P from GPU factors vs from oracle factors: <= 1e-12 relative
    (factors themselves are compared after aligning the joint sign of each term);
  * apply on the oracle's factors: global relative error over the batch
    <= 1e-12 (FP64), <= 1e-5 (FP32), <= 2e-2 (BF16);
  * setup + apply end to end (FP64): global <= 1e-12, and per element
    <= max(1e-12, 100 kappa(P) eps).
"""
import numpy as np
import pytest
import torch

import synth
from oracle.apply import dense_solve
from oracle.blocks import element_block
from oracle.ksvd import factor_array, factors_from_array, ksvd2d, ksvd3d, precond_matrix
from oracle.tables import tables

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def ctx():
    from paper_1704_04549_amd import kp
    c = kp.Ctx(0)
    yield c
    c.close()


def oracle_case(dim, n, E, seed, face):
    params = synth.draw_params(E, dim, seed, face=face)
    T = tables(n)
    blocks = np.stack([element_block(r, n, dim, T) for r in params])
    fo = [ksvd2d(A, n, 2) if dim == 2 else ksvd3d(A, n) for A in blocks]
    return params, blocks, fo


CASES = [  # dim, n, elements, seed, face
    (2, 8, 256, 1001, False),   # the full 2D p=7 workload
    (2, 16, 40, 1002, False),
    (3, 4, 30, 77, True),
    (3, 8, 12, 1003, True),
    (2, 20, 10, 1004, True),    # n > 16: the two-per-wave register inverses
    (2, 31, 3, 1005, False),
]


@pytest.mark.parametrize("dim,n,E,seed,face", CASES)
@pytest.mark.parametrize("explicit", [True, False])
def test_setup_and_apply_parity(ctx, dim, n, E, seed, face, explicit):
    from tests.gpu_util import align_sign, batch, rel, to_dev
    print(f"case dim={dim} n={n} E={E} seed={seed} explicit={explicit}", flush=True)
    params, blocks, fo = oracle_case(dim, n, E, seed, face)
    b = batch(params, dim, n)
    if explicit:
        gblocks = ctx.build_blocks(b)
        torch.cuda.synchronize()
        # rounding only: K = D^T W D sums n products whose terms grow like n^2
        # against the largest entry, so the bar grows like n^2 eps
        err = np.max(np.abs(gblocks.cpu().numpy() - blocks)) / np.max(np.abs(blocks))
        assert err <= max(1e-13, 2 * n * n * np.finfo(np.float64).eps), err
        b = batch(params, dim, n, blocks=gblocks)
    pc, st = ctx.setup(b, 2)
    f_gpu, s_gpu = ctx.get_factors(b, 2, pc)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0, st.cpu().numpy()
    f_gpu = f_gpu.cpu().numpy()
    s_gpu = s_gpu.cpu().numpy()
    for e in range(E):
        so = fo[e]["sigma"][:2] if dim == 2 else np.r_[fo[e]["sigma1"][0], fo[e]["sigma2"][:2]]
        sg = s_gpu[e, :2] if dim == 2 else s_gpu[e, :3]
        assert np.max(np.abs(sg / so - 1)) <= 1e-12, (e, sg, so)
        Pg = precond_matrix(factors_from_array(f_gpu[e], dim))
        Po = precond_matrix(fo[e])
        assert rel(Pg, Po) <= 1e-12, e
        Fo = factor_array(fo[e])
        if dim == 2:
            for j in range(2):
                a = align_sign(f_gpu[e, 2 * j], Fo[2 * j])
                sgn = np.sign(np.sum(f_gpu[e, 2 * j] * Fo[2 * j]))
                assert rel(a, Fo[2 * j]) <= 1e-10
                assert rel(sgn * f_gpu[e, 2 * j + 1], Fo[2 * j + 1]) <= 1e-10
    # apply on the oracle's factors
    rng = np.random.default_rng(seed + 7)
    r = rng.standard_normal((E, n ** dim))
    zref = np.stack([dense_solve(fo[e], r[e]) for e in range(E)])
    F_or = np.stack([factor_array(f) for f in fo])
    pco, st2 = ctx.setup_from_factors(b, 2, to_dev(F_or))
    rd = to_dev(r)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5), ("bf16", 2e-2), ("bf16x3", 1e-4)):
        z = ctx.apply(b, 2, pco, prec, rd)
        torch.cuda.synchronize()
        err = rel(z.cpu().numpy(), zref)
        print(f"  apply {prec} on oracle factors: {err:.3e}", flush=True)
        assert err <= tol, (prec, err)
    # end to end, FP64
    z = ctx.apply(b, 2, pc, "fp64", rd).cpu().numpy()
    assert rel(z, zref) <= 1e-12
    for e in range(E):
        kap = np.linalg.cond(precond_matrix(fo[e]))
        assert rel(z[e], zref[e]) <= max(1e-12, 100 * kap * EPS), e


def test_c4_matrix_free_sampled(ctx):
    """3D p=15 matrix-free setup at full size (4096 elements); sampled oracle check,
    and the FP32-z apply equal to the FP32 apply on every element."""
    from tests.gpu_util import batch, rel, to_dev
    w = synth.workload("c4_3d_p15")
    n, dim, E = 16, 3, w["num_elems"]
    print(f"case c4 full E={E}", flush=True)
    b = batch(w["params"], dim, n)
    pc, st = ctx.setup(b, 2)
    f_gpu, s_gpu = ctx.get_factors(b, 2, pc)
    rd = to_dev(w["rhs"][:, 0, :])
    z64 = ctx.apply(b, 2, pc, "fp64", rd)
    z32 = ctx.apply(b, 2, pc, "fp32", rd)
    # the launch the benchmark times (z stored in FP32): the same values on
    # every element
    z32f = ctx.apply_z32(b, 2, pc, "fp32", rd)
    torch.cuda.synchronize()
    assert torch.equal(z32f.double(), z32)
    assert int((st != 0).sum()) == 0
    f_gpu = f_gpu.cpu().numpy()
    T = tables(n)
    z64 = z64.cpu().numpy()
    z32 = z32.cpu().numpy()
    for e in (0, 1777, E - 1):
        A = element_block(w["params"][e], n, dim, T)
        fo = ksvd3d(A, n)
        so = np.r_[fo["sigma1"][0], fo["sigma2"][:2]]
        assert np.max(np.abs(s_gpu[e, :3].cpu().numpy() / so - 1)) <= 1e-12
        zref = dense_solve(fo, w["rhs"][e, 0])
        assert rel(z64[e], zref) <= 1e-11, e
        assert rel(z32[e], zref) <= 1e-4, e


def test_empty_batch(ctx):
    from tests.gpu_util import batch
    params = np.zeros((0, 16))
    b = batch(params, 2, 8)
    pc, st = ctx.setup(b, 2)
    z = ctx.apply(b, 2, pc, "fp64", torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert z.numel() == 0


def test_more_elements_than_setup_grid(ctx):
    """E above the persistent setup grid (2048 workgroups): every element is set up."""
    from tests.gpu_util import batch
    E = 2051
    params = synth.draw_params(E, 2, 55)
    b = batch(params, 2, 6)
    pc, st = ctx.setup(b, 2)
    f, s = ctx.get_factors(b, 2, pc)
    torch.cuda.synchronize()
    s = s.cpu().numpy()
    for e in (0, 2047, 2048, 2050):
        so = ksvd2d(element_block(params[e], 6, 2), 6, 2)["sigma"][:2]
        assert np.max(np.abs(s[e, :2] / so - 1)) <= 1e-12


@pytest.mark.parametrize("dim,nrhs", [(3, 2), (2, 8), (2, 20), (2, 1)])
def test_mfma16_apply_matches_generic_and_oracle(ctx, dim, nrhs, monkeypatch):
    """The n = 16 matrix-core apply against the generic kernel and the oracle, all precisions
    (2D with 20 right-hand sides exercises a ragged second group of slices, with one a group
    of one)."""
    from paper_1704_04549_amd import kp
    from tests.gpu_util import batch, rel, to_dev
    n, E = 16, 12
    print(f"mfma16 dim={dim} nrhs={nrhs}", flush=True)
    params = synth.draw_params(E, dim, 321 + dim, face=(dim == 3))
    b = batch(params, dim, n)
    pc, st = ctx.setup(b, 2)
    r = np.random.default_rng(5).standard_normal((E, nrhs, n ** dim))
    rd = to_dev(r)
    monkeypatch.setenv("KP_APPLY_GENERIC", "1")
    gctx = kp.Ctx(0)
    f_gpu, _ = ctx.get_factors(b, 2, pc)
    fo = [factors_from_array(f, dim) for f in f_gpu.cpu().numpy()]
    zref = np.stack([dense_solve(fo[e], r[e]) for e in range(E)])
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5), ("bf16", 2e-2), ("bf16x3", 1e-4)):
        zm = ctx.apply(b, 2, pc, prec, rd)
        zg = gctx.apply(b, 2, pc, prec, rd)
        torch.cuda.synchronize()
        em, eg = rel(zm.cpu().numpy(), zref), rel(zg.cpu().numpy(), zref)
        print(f"  {prec}: mfma {em:.2e} generic {eg:.2e}", flush=True)
        assert em <= tol and eg <= tol
    gctx.close()


def test_c4_stratified_64_elements(ctx):
    """3D p = 15 at full size (4096 elements): on 64 elements spread evenly
    over the batch, singular values within 1e-12 of the oracle's full SVDs and
    the global relative error of z = P^{-1} r over those elements within
    1e-12 (FP64), 1e-5 (FP32), 1e-4 (split BF16) and 2e-2 (BF16) of the
    oracle's solves (tests/golden/c4_sampled.npz, written by
    tests/golden/make_c4_sampled.py from oracle/ alone)."""
    import os

    from tests.gpu_util import batch, rel, to_dev
    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c4_sampled.npz"))
    idx, sig, zref = g["idx"], g["sigma"], g["z"]
    w = synth.workload("c4_3d_p15")
    print(f"case c4 stratified {len(idx)} of {w['num_elems']}", flush=True)
    b = batch(w["params"], 3, 16)
    pc, st = ctx.setup(b, 2)
    _, s_gpu = ctx.get_factors(b, 2, pc)
    s_gpu = s_gpu.cpu().numpy()[idx, :3]
    assert np.max(np.abs(s_gpu / sig - 1)) <= 1e-12
    rd = to_dev(w["rhs"][:, 0, :])
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5), ("bf16x3", 1e-4), ("bf16", 2e-2)):
        z = ctx.apply(b, 2, pc, prec, rd)
        torch.cuda.synchronize()
        err = rel(z.cpu().numpy()[idx], zref)
        print(f"  {prec}: {err:.2e}", flush=True)
        assert err <= tol, (prec, err)
