"""FGMRES with every restart cycle replayed as one HIP graph.

The cycle's graph holds the eager solve's kernels for each Arnoldi step in
the same order (the next basis vector normalised on the device with the same
arithmetic), and the host stops at the same column, so the iteration count
and the solution must be bit-identical; the graph is replayed once per
restart cycle, with the driver's own eager work and synchronisations in
between, and the restart lengths below force many cycles.  Covers the
uniform coupled operator (KSVD and block-Jacobi preconditioners), a mixed
batch and a systems batch.
"""
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1704_04549_amd import kp
    c = kp.Ctx(0)
    yield c
    c.set_option(kp.KP_OPT_FGMRES_GRAPHS, 0)
    c.close()


def run(ctx, graphs, fn):
    import torch

    from paper_1704_04549_amd import kp
    ctx.set_option(kp.KP_OPT_FGMRES_GRAPHS, 1 if graphs else 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


@pytest.mark.parametrize("dim,n,mesh,restart", [(2, 8, 16, 5), (3, 4, 6, 7)])
def test_graph_fgmres_identical_to_eager(ctx, dim, n, mesh, restart):
    from paper_1704_04549_amd import kp
    from tests.gpu_util import batch, to_dev
    print(f"graphs dim={dim} n={n} mesh={mesh} restart={restart}", flush=True)
    params, nbr = synth.mesh_params(mesh, dim, 51)
    E = mesh ** dim
    b = batch(params, dim, n, nbr=nbr)
    rhs = to_dev(np.random.default_rng(5).standard_normal((E, n ** dim)))
    pc, _ = ctx.setup(b, 2)
    bd = batch(params, dim, n, blocks=ctx.build_blocks(b), nbr=nbr)
    lu, piv, _ = ctx.blockjacobi_exact(bd)
    cases = (("ksvd fp32", dict(pc_kind=kp.KP_PC_KSVD, pc_data=pc, pc_prec="fp32")),
             ("bj", dict(pc_kind=kp.KP_PC_BJ, pc_data=lu, pc_aux=piv)))
    for name, kw in cases:
        f = lambda: ctx.fgmres(b, rhs, restart=restart, rtol=1e-10, maxit=2000, **kw)
        e, te = run(ctx, False, f)
        g, tg = run(ctx, True, f)
        print(f"  {name}: iters {e['iters']} / {g['iters']}, eager {te * 1e3:.1f} ms, graphs {tg * 1e3:.1f} ms",
              flush=True)
        assert e["converged"] and g["converged"]
        assert e["iters"] == g["iters"] and e["iters"] > 3 * restart
        assert np.array_equal(e["x"].cpu().numpy(), g["x"].cpu().numpy())


def test_graph_fgmres_mixed_batch(ctx):
    from paper_1704_04549_amd import kp
    from tests.gpu_util import to_dev
    dims, ns, recs = synth.mixed_batch(300, 30, seed=77)
    plan = kp.MixedPlan(ctx, dims, ns, to_dev(recs))
    pc, _ = plan.setup()
    rhs = to_dev(np.random.default_rng(6).standard_normal(plan.vec_len))
    f = lambda: plan.fgmres(rhs, pc_kind=kp.KP_PC_KSVD, precond=pc, pc_prec="fp32", restart=6)
    e, te = run(ctx, False, f)
    g, tg = run(ctx, True, f)
    print(f"  mixed: iters {e['iters']} / {g['iters']}, eager {te * 1e3:.1f} ms, graphs {tg * 1e3:.1f} ms",
          flush=True)
    assert e["converged"] and e["iters"] == g["iters"]
    assert np.array_equal(e["x"].cpu().numpy(), g["x"].cpu().numpy())
    plan.close()


def test_graph_fgmres_systems(ctx):
    from oracle import systems
    from paper_1704_04549_amd import kp
    from tests.gpu_util import to_dev
    nc, n, E = 4, 6, 40
    sd = synth.systems_elements(E, nc, seed=12)
    A = to_dev(np.stack([systems.element_block(sd, e, n) for e in range(E)]))
    sb = kp.SysBatch(nc, n, A)
    pc, _ = ctx.setup_sys(sb)
    rhs = to_dev(np.random.default_rng(8).standard_normal(E * nc * n * n))
    f = lambda: ctx.fgmres_sys(sb, rhs, pc_kind=kp.KP_PC_KSVD, pc_data=pc, pc_prec="fp32", restart=4)
    e, te = run(ctx, False, f)
    g, tg = run(ctx, True, f)
    print(f"  systems: iters {e['iters']} / {g['iters']}, eager {te * 1e3:.1f} ms, graphs {tg * 1e3:.1f} ms",
          flush=True)
    assert e["converged"] and e["iters"] == g["iters"] and e["iters"] > 8
    assert np.array_equal(e["x"].cpu().numpy(), g["x"].cpu().numpy())

