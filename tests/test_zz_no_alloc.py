"""kp_setup_noalloc (static scratch, no device allocation) against kp_setup.

Two calls in a row on one context, the second with a smaller batch (the
scratch keeps the first call's contents): factors, singular values, element
status and the applied preconditioner are bit-identical to kp_setup's.
"""
import numpy as np
import pytest
import torch

import synth
from paper_1704_04549_amd import kp

from gpu_util import DEV, batch, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    # dim, n, explicit blocks, rank, first E, second E
    (3, 16, False, 2, 300, 37),
    (2, 16, True, 2, 40, 9),
    (2, 8, False, 3, 70, 5),
    (3, 8, True, 2, 20, 3),
]


def _batch(ctx, dim, n, expl, E, seed):
    params = synth.draw_params(E, dim, seed=seed, face=dim == 3)
    b = batch(params, dim, n)
    if expl:
        blocks = ctx.build_blocks(b)
        b = batch(params, dim, n, blocks=blocks)
        b._keep = blocks
    return b


@pytest.mark.parametrize("dim,n,expl,rank,E1,E2", CASES)
def test_noalloc_setup_matches_setup(dim, n, expl, rank, E1, E2):
    print(f"noalloc dim={dim} n={n} explicit={expl} rank={rank} E={E1},{E2}", flush=True)
    ctx = kp.Ctx(0)
    try:
        for call, E in enumerate((E1, E2)):
            b = _batch(ctx, dim, n, expl, E, seed=500 + 10 * call + dim)
            nbytes = ctx.precond_bytes(dim, n, rank, E)
            ref, st_ref = ctx.setup(b, rank)
            pc = torch.empty(nbytes, dtype=torch.uint8, device=DEV)
            st = torch.full((E,), -7, dtype=torch.int32, device=DEV)
            ctx.setup_noalloc(b, rank, pc, st)
            torch.cuda.synchronize()
            f_ref, s_ref = ctx.get_factors(b, rank, ref)
            f, s = ctx.get_factors(b, rank, pc)
            assert torch.equal(st.cpu(), st_ref.cpu())
            assert torch.equal(f.cpu(), f_ref.cpu()), "factors differ"
            assert torch.equal(s.cpu(), s_ref.cpu()), "singular values differ"
            r = to_dev(np.random.default_rng(77 + call).standard_normal((E, 1, n ** dim)))
            for prec in ("fp64", "fp32"):
                z_ref = ctx.apply(b, rank, ref, prec, r)
                z = ctx.apply(b, rank, pc, prec, r)
                torch.cuda.synchronize()
                assert torch.equal(z.cpu(), z_ref.cpu()), prec
    finally:
        ctx.close()
