"""The 3D apply for n <= 8 with one wave per (element, right-hand side)
(KP_OPT_APPLY_SMALL3, the default) against the oracle and against the generic
per-element kernel it replaces.

Bars: z = P^{-1} r against the oracle's dense solve of P at 1e-12 (FP64),
1e-5 (FP32), 1e-4 (split BF16), 2e-2 (BF16), global relative, for n = 2, 3,
5, 7, 8 on ragged batches with two right-hand sides, on records with faces (the
Schur forms then hold 2 x 2 blocks); the two kernels agree to 1e-13 (FP64)
and 1e-6 (the FP32 forms) relatively on every element; the FP32-stored form
(kp_apply_z32) equals the FP64-stored one's FP32 values; with split axes
(KP_OPT_SPLIT_AXIS) the kernels agree as well.
"""
import numpy as np
import pytest

import synth
from oracle.apply import dense_solve
from oracle.blocks import element_block
from oracle.ksvd import ksvd3d
from oracle.tables import tables

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-4, "bf16": 2e-2}
AGREE = {"fp64": 1e-13, "fp32": 1e-6, "bf16x3": 1e-6, "bf16": 1e-6}


@pytest.fixture(scope="module")
def ctx():
    from paper_1704_04549_amd import kp
    c = kp.Ctx(0)
    yield c
    c.set_option(kp.KP_OPT_APPLY_SMALL3, 1)
    c.set_option(kp.KP_OPT_SPLIT_AXIS, 0)
    c.close()


@pytest.mark.parametrize("n,E", [(2, 29), (3, 41), (5, 23), (7, 17), (8, 19)])
def test_small3_matches_oracle_and_generic(ctx, n, E):
    import torch

    from paper_1704_04549_amd import kp
    from tests.gpu_util import batch, rel, to_dev
    print(f"small3 n={n} E={E}", flush=True)
    params = synth.draw_params(E, 3, 500 + n, face=True)
    b = batch(params, 3, n)
    pc, st = ctx.setup(b, 2)
    torch.cuda.synchronize()
    assert int((st != 0).sum()) == 0
    r = np.random.default_rng(n).standard_normal((E, 2, n ** 3))
    rd = to_dev(r)
    T = tables(n)
    zref = np.stack([dense_solve(ksvd3d(element_block(params[e], n, 3, T), n), r[e]) for e in range(E)])
    for prec in TOL:
        zs = ctx.apply(b, 2, pc, prec, rd).cpu().numpy()
        ctx.set_option(kp.KP_OPT_APPLY_SMALL3, 0)
        zg = ctx.apply(b, 2, pc, prec, rd).cpu().numpy()
        ctx.set_option(kp.KP_OPT_APPLY_SMALL3, 1)
        err = rel(zs, zref)
        worst = max(rel(zs[e], zg[e]) for e in range(E))
        print(f"  {prec}: vs oracle {err:.2e}, vs generic {worst:.2e}", flush=True)
        assert err <= TOL[prec]
        assert worst <= AGREE[prec]
        if prec != "fp64":
            z32 = ctx.apply_z32(b, 2, pc, prec, rd).cpu().numpy()
            assert np.array_equal(z32, zs.astype(np.float32))


def test_small3_split_axes_match_generic(ctx):
    import torch

    from paper_1704_04549_amd import kp
    from tests.gpu_util import batch, rel, to_dev
    n, E = 6, 31
    ctx.set_option(kp.KP_OPT_SPLIT_AXIS, 1)
    try:
        params = synth.draw_params(E, 3, 77, face=True)
        b = batch(params, 3, n)
        pc, st = ctx.setup(b, 2)
        axes = ctx.get_axes(b, 2, pc).cpu().numpy()
        torch.cuda.synchronize()
        assert int((st != 0).sum()) == 0 and len(set(axes.tolist())) > 1
        rd = to_dev(np.random.default_rng(3).standard_normal((E, n ** 3)))
        for prec in ("fp64", "fp32"):
            zs = ctx.apply(b, 2, pc, prec, rd).cpu().numpy()
            ctx.set_option(kp.KP_OPT_APPLY_SMALL3, 0)
            zg = ctx.apply(b, 2, pc, prec, rd).cpu().numpy()
            ctx.set_option(kp.KP_OPT_APPLY_SMALL3, 1)
            assert max(rel(zs[e], zg[e]) for e in range(E)) <= AGREE[prec]
    finally:
        ctx.set_option(kp.KP_OPT_SPLIT_AXIS, 0)
