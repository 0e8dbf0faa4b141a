"""The apply with z stored in FP32 (kp_apply_z32) and the FP32 FGMRES basis.

In FP32, BF16 and split BF16 the rank-2 apply ends in FP32 arithmetic, so
its outputs are FP32 numbers: kp_apply_z32 must store exactly the values
kp_apply stores as FP64 (bit-identical after widening), on every kernel that
serves the apply (the 3D and 2D matrix-core kernels for n = 16, the generic
kernel otherwise, and the generic kernel for n = 16 when the matrix-core path
is switched off), with ragged element counts and a partial group of
right-hand sides.  FP64 and rank 3 are refused.  FGMRES with the FP32 basis
must give the same iterations and a bit-identical solution as with an FP64
basis, eager and as HIP graphs (over a fixed budget of at most 300 steps).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1704_04549_amd import kp
    c = kp.Ctx(0)
    yield c
    c.set_option(kp.KP_OPT_APPLY_MFMA16, 1)
    c.set_option(kp.KP_OPT_FGMRES_Z32, 1)
    c.set_option(kp.KP_OPT_FGMRES_GRAPHS, 0)
    c.close()


@pytest.mark.parametrize("dim,n,E,nrhs,mfma", [(3, 16, 37, 1, 1), (3, 16, 5, 3, 1), (3, 16, 9, 2, 0), (2, 16, 21, 8, 1),
                                                (2, 16, 13, 19, 1), (2, 16, 7, 3, 1), (2, 8, 45, 3, 1), (3, 5, 33, 1, 1),
                                                (2, 31, 6, 2, 1)])
def test_apply_z32_matches_apply(ctx, dim, n, E, nrhs, mfma):
    import torch

    from paper_1704_04549_amd import kp
    from tests.gpu_util import batch, to_dev
    print(f"z32 apply dim={dim} n={n} E={E} nrhs={nrhs} mfma={mfma}", flush=True)
    ctx.set_option(kp.KP_OPT_APPLY_MFMA16, mfma)
    params = synth.draw_params(E, dim, 900 + n, face=True)
    b = batch(params, dim, n)
    pc, st = ctx.setup(b, 2)
    r = to_dev(np.random.default_rng(n + E).standard_normal((E, nrhs, n ** dim)))
    for prec in ("fp32", "bf16", "bf16x3"):
        z64 = ctx.apply(b, 2, pc, prec, r)
        z32 = ctx.apply_z32(b, 2, pc, prec, r)
        torch.cuda.synchronize()
        assert z32.dtype == torch.float32
        assert torch.equal(z32.double(), z64), prec
        assert bool(torch.isfinite(z64).all())
    ctx.set_option(kp.KP_OPT_APPLY_MFMA16, 1)
    assert int((st != 0).sum()) == 0


def test_apply_z32_refuses_fp64_and_rank3(ctx):
    from paper_1704_04549_amd import kp
    from tests.gpu_util import batch, to_dev
    params = synth.draw_params(4, 2, 31, face=True)
    b = batch(params, 2, 8)
    r = to_dev(np.random.default_rng(3).standard_normal((4, 64)))
    pc2, _ = ctx.setup(b, 2)
    with pytest.raises(kp.KpError) as ei:
        ctx.apply_z32(b, 2, pc2, "fp64", r)
    assert ei.value.status == kp.KP_ERR_UNSUPPORTED
    pc3, _ = ctx.setup(b, 3)
    with pytest.raises(kp.KpError) as ei:
        ctx.apply_z32(b, 3, pc3, "fp32", r)
    assert ei.value.status == kp.KP_ERR_UNSUPPORTED


@pytest.mark.parametrize("dim,n,mesh,restart,prec,explicit", [(3, 16, 3, 10, "fp32", False),
                                                              (2, 8, 12, 6, "bf16x3", False),
                                                              (3, 6, 5, 8, "bf16", False),
                                                              (2, 8, 10, 7, "fp32", True)])
def test_fgmres_z32_basis_identical(ctx, dim, n, mesh, restart, prec, explicit):
    import torch

    from paper_1704_04549_amd import kp
    from tests.gpu_util import batch, to_dev
    print(f"z32 fgmres dim={dim} n={n} mesh={mesh} restart={restart} {prec} explicit={explicit}", flush=True)
    params, nbr = synth.mesh_params(mesh, dim, 61)
    E = mesh ** dim
    b = batch(params, dim, n, nbr=nbr)
    if explicit:
        # the operator reads the explicit blocks (and the FP32 basis through them)
        b = batch(params, dim, n, blocks=ctx.build_blocks(b), nbr=nbr)
    rhs = to_dev(np.random.default_rng(8).standard_normal((E, n ** dim)))
    pc, _ = ctx.setup(b, 2)
    out = {}
    for graphs in (0, 1):
        ctx.set_option(kp.KP_OPT_FGMRES_GRAPHS, graphs)
        for z32 in (0, 1):
            ctx.set_option(kp.KP_OPT_FGMRES_Z32, z32)
            o = ctx.fgmres(b, rhs, kp.KP_PC_KSVD, 2, pc, None, prec, restart=restart, rtol=1e-10, maxit=300)
            torch.cuda.synchronize()
            out[(graphs, z32)] = (o["iters"], o["converged"], o["x"].cpu().numpy())
            print(f"  graphs={graphs} z32={z32}: {o['iters']} iterations", flush=True)
    ctx.set_option(kp.KP_OPT_FGMRES_GRAPHS, 0)
    ctx.set_option(kp.KP_OPT_FGMRES_Z32, 1)
    # several restart cycles (each ends in the combine x += Z y); convergence
    # itself is not required, the solves must agree bit for bit
    ref = out[(0, 0)]
    assert ref[0] > 2 * restart
    for key, (it, conv, x) in out.items():
        assert it == ref[0] and conv == ref[1], key
        assert np.array_equal(x, ref[2]), key
