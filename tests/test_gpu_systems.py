"""Blocks of nc-component systems (2D; nc n x nc n first factors) on the GPU
through the C ABI, against the oracle (oracle/systems.py).

Bars: sigma_1, sigma_2 within 1e-12 and every factor within 1e-10 (relative,
sign included: the pair is signed so that A_j's largest-magnitude entry is
positive) of the oracle's full SVD of R(A); z = P^{-1} r within 1e-12 (FP64)
and 5e-5 (FP32) of the oracle's dense solve of P, two right-hand sides, ragged
batch sizes that span several workgroups of the persistent setup grid.  The
"small" variant (the nc diagonal component blocks, Sec. 5.6) runs through
the scalar explicit-block setup and apply against the oracle's KSVD of each
component block.  The block builder against the oracle's assembly (1e-14),
the block-diagonal operator and exact block Jacobi against numpy, and
FGMRES(30) iteration counts against the oracle's FGMRES (within one).
"""
import numpy as np
import pytest

import synth
from oracle import systems
from oracle.apply import dense_solve
from oracle.ksvd import ksvd2d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1704_04549_amd import kp
    c = kp.Ctx(0)
    yield c
    c.close()


def sys_blocks(nc, n, E, seed):
    sd = synth.systems_elements(E, nc, seed=seed)
    return np.stack([systems.element_block(sd, e, n) for e in range(E)])


@pytest.mark.parametrize("nc,n,E", [(1, 5, 3), (2, 4, 7), (4, 4, 5), (4, 8, 3), (5, 6, 4), (3, 8, 6), (2, 16, 2),
                                    (1, 32, 1)])
def test_systems_setup_and_apply_match_oracle(ctx, nc, n, E):
    from paper_1704_04549_amd import kp
    from tests.gpu_util import rel, to_dev
    print(f"systems nc={nc} n={n} E={E}", flush=True)
    m = nc * n
    A = sys_blocks(nc, n, E, seed=500 + 7 * nc + n)
    sb = kp.SysBatch(nc, n, to_dev(A))
    pc, st = ctx.setup_sys(sb)
    F, sg = ctx.get_factors_sys(sb, pc)
    F, sg, st = F.cpu().numpy(), sg.cpu().numpy(), st.cpu().numpy()
    r = np.random.default_rng(nc * 100 + n).standard_normal((E, 2, m * n))
    z64 = ctx.apply_sys(sb, pc, "fp64", to_dev(r)).cpu().numpy()
    z32 = ctx.apply_sys(sb, pc, "fp32", to_dev(r)).cpu().numpy()
    for e in range(E):
        f = systems.ksvd_system(A[e], nc, n, 2)
        assert st[e] == 0
        assert np.max(np.abs(sg[e, :2] / f["sigma"][:2] - 1)) <= 1e-12
        off = 0
        for j in range(2):
            assert rel(F[e, off:off + m * m], f["A"][j]) <= 1e-10
            assert rel(F[e, off + m * m:off + m * m + n * n], f["B"][j]) <= 1e-10
            off += m * m + n * n
        for k in range(2):
            zr = dense_solve(f, r[e, k])
            assert rel(z64[e, k], zr) <= 1e-12
            assert rel(z32[e, k], zr) <= 5e-5


def test_systems_edge_cases(ctx):
    import torch

    from paper_1704_04549_amd import kp
    from tests.gpu_util import to_dev
    assert ctx.sys_precond_bytes(4, 9, 1) == 0        # nc n = 36 > 32
    assert ctx.sys_precond_bytes(1, 1, 1) == 0        # n < 2
    empty = kp.SysBatch(2, 4, torch.empty((0, 32, 32), dtype=torch.float64, device="cuda"))
    pc, _ = ctx.setup_sys(empty)
    z = ctx.apply_sys(empty, pc, "fp64", torch.empty(0, dtype=torch.float64, device="cuda"))
    assert z.numel() == 0
    A = sys_blocks(2, 4, 1, seed=9)
    sb = kp.SysBatch(2, 4, to_dev(A))
    pc, st = ctx.setup_sys(sb)
    with pytest.raises(kp.KpError) as ei:
        ctx.apply_sys(sb, pc, "bf16", to_dev(np.ones(32)))
    assert ei.value.status == kp.KP_ERR_UNSUPPORTED
    bad = kp.SysBatch(4, 9, num_elems=1)
    with pytest.raises(kp.KpError) as ei:
        ctx.apply_sys(bad, pc, "fp64", to_dev(np.ones(324)))
    assert ei.value.status == kp.KP_ERR_ARG


@pytest.mark.parametrize("nc,n", [(3, 5), (4, 8)])
def test_small_component_blocks_through_scalar_setup(ctx, nc, n):
    """The small block-Jacobi variant: each component's n^2 x n^2 diagonal
    block as a scalar explicit block (kp_setup, kp_apply) against the oracle's
    KSVD of that block."""
    from tests.gpu_util import align_sign, batch, rel, to_dev
    print(f"systems small nc={nc} n={n}", flush=True)
    E = 3
    A = sys_blocks(nc, n, E, seed=40 + nc)
    small = np.stack([b for e in range(E) for b in systems.small_blocks(A[e], nc, n)])
    b = batch(np.zeros((E * nc, 16)), 2, n, blocks=small)
    pc, st = ctx.setup(b, 2)
    F, sg = ctx.get_factors(b, 2, pc)
    F, sg = F.cpu().numpy(), sg.cpu().numpy()
    assert int(st.abs().sum()) == 0
    r = np.random.default_rng(3).standard_normal((E * nc, n * n))
    z = ctx.apply(b, 2, pc, "fp64", to_dev(r)).cpu().numpy()
    for i in range(E * nc):
        f = ksvd2d(small[i], n, 2)
        assert np.max(np.abs(sg[i, :2] / f["sigma"][:2] - 1)) <= 1e-12
        for j in range(2):
            assert rel(align_sign(F[i, 2 * j], f["A"][j]), f["A"][j]) <= 1e-10
        assert rel(z[i], dense_solve(f, r[i])) <= 1e-12


@pytest.mark.parametrize("nc,n,E", [(2, 4, 5), (4, 8, 3), (3, 5, 4), (1, 6, 2)])
def test_build_sys_blocks_matches_oracle(ctx, nc, n, E):
    """kp_build_sys_blocks from the packed records against the oracle's
    assembly of the same weak form (faces on and off)."""
    from tests.gpu_util import to_dev
    print(f"systems blocks nc={nc} n={n} E={E}", flush=True)
    for face in (True, False):
        sd = synth.systems_elements(E, nc, seed=70 + nc + n, face=face)
        recs = synth.systems_records(sd)
        A = ctx.build_sys_blocks(nc, n, to_dev(recs)).cpu().numpy()
        for e in range(E):
            Ar = systems.element_block(sd, e, n)
            assert np.max(np.abs(A[e] - Ar)) <= 1e-14 * np.abs(Ar).max()


def test_sys_operator_and_block_jacobi(ctx):
    from paper_1704_04549_amd import kp
    from tests.gpu_util import rel, to_dev
    nc, n, E = 4, 6, 5
    A = sys_blocks(nc, n, E, seed=81)
    sb = kp.SysBatch(nc, n, to_dev(A))
    x = np.random.default_rng(2).standard_normal((E, nc * n * n))
    y = ctx.sys_operator_apply(sb, to_dev(x)).cpu().numpy()
    assert rel(y, np.einsum("eij,ej->ei", A, x)) <= 1e-14
    lu, piv, st = ctx.sys_blockjacobi_exact(sb)
    assert int(st[:E].abs().sum()) == 0
    r = to_dev(x)
    out = ctx.fgmres_sys(sb, r, pc_kind=kp.KP_PC_BJ, pc_data=lu, pc_aux=piv, rtol=1e-12)
    zr = np.stack([np.linalg.solve(A[e], x[e]) for e in range(E)])
    assert out["converged"] and out["iters"] <= 2
    assert rel(out["x"].cpu().numpy(), zr) <= 1e-10


@pytest.mark.parametrize("nc,n,E,face", [(4, 6, 6, True), (4, 8, 4, True), (2, 8, 5, False)])
def test_sys_fgmres_iterations_match_oracle(ctx, nc, n, E, face):
    """FGMRES(30) to 1e-10 on the block-diagonal systems operator with the
    systems KSVD preconditioner: the GPU's FP64 count within one of the
    oracle's FGMRES with the oracle's preconditioner (dense solve of P), the
    FP32 apply within one of the FP64 count, the solution against a dense
    solve."""
    from oracle.krylov import fgmres
    from paper_1704_04549_amd import kp
    from tests.gpu_util import rel, to_dev
    print(f"systems fgmres nc={nc} n={n} E={E} face={face}", flush=True)
    sd = synth.systems_elements(E, nc, seed=90 + n, face=face)
    A = np.stack([systems.element_block(sd, e, n) for e in range(E)])
    N = nc * n * n
    rhs = np.random.default_rng(n).standard_normal(E * N)
    fs = [systems.ksvd_system(A[e], nc, n, 2) for e in range(E)]
    Aop = lambda v: np.einsum("eij,ej->ei", A, v.reshape(E, N)).ravel()
    Mop = lambda v: np.concatenate([dense_solve(fs[e], v.reshape(E, N)[e]) for e in range(E)])
    _, it_ref, _, conv = fgmres(Aop, Mop, rhs, m=30, rtol=1e-10)
    assert conv
    sb = kp.SysBatch(nc, n, to_dev(A))
    pc, st = ctx.setup_sys(sb)
    assert int(st.abs().sum()) == 0
    r = to_dev(rhs)
    o64 = ctx.fgmres_sys(sb, r, pc_kind=kp.KP_PC_KSVD, pc_data=pc, pc_prec="fp64")
    o32 = ctx.fgmres_sys(sb, r, pc_kind=kp.KP_PC_KSVD, pc_data=pc, pc_prec="fp32")
    print(f"  iters oracle {it_ref} fp64 {o64['iters']} fp32 {o32['iters']}", flush=True)
    assert o64["converged"] and o32["converged"]
    assert abs(o64["iters"] - it_ref) <= 1
    assert o32["iters"] <= o64["iters"] + 1
    xr = np.concatenate([np.linalg.solve(A[e], rhs.reshape(E, N)[e]) for e in range(E)])
    assert rel(o64["x"].cpu().numpy(), xr) <= 1e-8
