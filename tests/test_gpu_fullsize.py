"""GPU parity at the full sizes of the 2D p = 15 and 3D p = 7 workloads.

The whole batch runs on the GPU in the library's own launch configuration;
the oracle checks sampled elements one by one (its dense per-element forms),
and properties that hold at any size are checked on the whole batch.
Bars per sampled element: sigma relative <= 1e-12; apply against the
oracle's dense solve <= 1e-11 (FP64), <= 1e-4 (FP32), <= 5e-2 (BF16),
<= 1e-3 (split BF16); rank 3 (FP64) <= max(1e-11, 100 kappa(P3) eps); the
coupled operator <= 1e-12 of || |G_e| |x| ||.  Whole batch: every element's
setup status is zero; on the coupled 3D p = 7 system FGMRES(30) with the
FP32 apply ends within 10% of the FP64 apply's true residual after a fixed
budget (the rank-2 preconditioner does not converge there at full size), and
on a 4^3 mesh of the same generator both reach 1e-10 with FP32 within one
iteration of FP64.
"""
import numpy as np
import pytest

import synth
from oracle.apply import dense_solve
from oracle.blocks import element_block
from oracle.ksvd import ksvd2d, ksvd3d, precond_matrix
from oracle.operator import coupling_blocks
from oracle.tables import tables

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def ctx():
    from paper_1704_04549_amd import kp
    c = kp.Ctx(0)
    yield c
    c.close()


def test_c2_full_rank2_sampled(ctx):
    import torch

    from tests.gpu_util import batch, rel, to_dev
    w = synth.workload("c2_2d_p15")
    n, dim, E, nrhs = 16, 2, w["num_elems"], w["nrhs"]
    print(f"case c2 full E={E} nrhs={nrhs} rank 2", flush=True)
    b = batch(w["params"], dim, n)
    pc, st = ctx.setup(b, 2)
    _, s_gpu = ctx.get_factors(b, 2, pc)
    rd = to_dev(w["rhs"])
    zs = {p: ctx.apply(b, 2, pc, p, rd) for p in ("fp64", "fp32", "bf16", "bf16x3")}
    torch.cuda.synchronize()
    assert int((st != 0).sum()) == 0
    s_gpu = s_gpu.cpu().numpy()
    zs = {p: z.cpu().numpy() for p, z in zs.items()}
    T = tables(n)
    for e in (0, 7777, E - 1):
        fo = ksvd2d(element_block(w["params"][e], n, dim, T), n, 2)
        assert np.max(np.abs(s_gpu[e, :2] / fo["sigma"][:2] - 1)) <= 1e-12, e
        zref = dense_solve(fo, w["rhs"][e])
        for p, tol in (("fp64", 1e-11), ("fp32", 1e-4), ("bf16", 5e-2), ("bf16x3", 1e-3)):
            err = rel(zs[p][e], zref)
            print(f"  e={e} {p}: {err:.2e}", flush=True)
            assert err <= tol, (e, p, err)


def test_c2_full_rank3_sampled(ctx):
    import torch

    from tests.gpu_util import batch, rel, to_dev
    w = synth.workload("c2_2d_p15")
    n, dim, E = 16, 2, w["num_elems"]
    print(f"case c2 full E={E} rank 3", flush=True)
    b = batch(w["params"], dim, n)
    pc, st = ctx.setup(b, 3)
    _, s_gpu = ctx.get_factors(b, 3, pc)
    rd = to_dev(w["rhs"])
    zs = {p: ctx.apply(b, 3, pc, p, rd) for p in ("fp64", "fp32", "bf16", "bf16x3")}
    torch.cuda.synchronize()
    assert int((st != 0).sum()) == 0
    s_gpu = s_gpu.cpu().numpy()
    zs = {p: z.cpu().numpy() for p, z in zs.items()}
    T = tables(n)
    for e in (1, 9000, E - 2):
        fo = ksvd2d(element_block(w["params"][e], n, dim, T), n, 3)
        assert np.max(np.abs(s_gpu[e, :3] / fo["sigma"][:3] - 1)) <= 1e-12, e
        zref = dense_solve(fo, w["rhs"][e])
        kap = np.linalg.cond(precond_matrix(fo))
        err = rel(zs["fp64"][e], zref)
        print(f"  e={e}: {err:.2e} (kappa {kap:.1e})", flush=True)
        assert err <= max(1e-11, 100 * kap * EPS), e
        # the reduced-precision series, to the rank-2 full-size bars
        for p, tol in (("fp32", 1e-4), ("bf16", 5e-2), ("bf16x3", 1e-3)):
            err = rel(zs[p][e], zref)
            print(f"  e={e} {p}: {err:.2e}", flush=True)
            assert err <= tol, (e, p, err)


def test_c3_full_sampled_and_fgmres(ctx):
    import torch

    from paper_1704_04549_amd import kp
    from tests.gpu_util import batch, rel, to_dev
    w = synth.workload("c3_3d_p7")
    n, dim, E = 8, 3, w["num_elems"]
    print(f"case c3 full E={E} coupled", flush=True)
    b = batch(w["params"], dim, n, nbr=w["nbr"])
    pc, st = ctx.setup(b, 2)
    _, s_gpu = ctx.get_factors(b, 2, pc)
    rhs = w["rhs"][:, 0, :]
    rd = to_dev(rhs)
    z64 = ctx.apply(b, 2, pc, "fp64", rd)
    z32 = ctx.apply(b, 2, pc, "fp32", rd)
    xr = np.random.default_rng(7).standard_normal((E, n ** dim))
    y = ctx.operator_apply(b, to_dev(xr))
    torch.cuda.synchronize()
    assert int((st != 0).sum()) == 0
    s_gpu = s_gpu.cpu().numpy()
    z64, z32, y = z64.cpu().numpy(), z32.cpu().numpy(), y.cpu().numpy()
    T = tables(n)
    for e in (0, 12345, E - 1):
        A = element_block(w["params"][e], n, dim, T)
        fo = ksvd3d(A, n)
        so = np.r_[fo["sigma1"][0], fo["sigma2"][:2]]
        assert np.max(np.abs(s_gpu[e, :3] / so - 1)) <= 1e-12, e
        zref = dense_solve(fo, rhs[e])
        assert rel(z64[e], zref) <= 1e-11, e
        assert rel(z32[e], zref) <= 1e-4, e
        # the coupled operator on this element's rows
        ye = A @ xr[e]
        ya = np.abs(A) @ np.abs(xr[e])
        for ax in range(dim):
            for col, C in coupling_blocks(w["params"][e], ax, dim, T):
                xn = xr[w["nbr"][e, col]]
                ye = ye + C @ xn
                ya = ya + np.abs(C) @ np.abs(xn)
        assert np.linalg.norm(y[e] - ye) <= 1e-12 * np.linalg.norm(ya), e
    # FGMRES(30) on the whole coupled system with a fixed budget: the rank-2
    # KSVD preconditioner does not make this system converge at this size
    # (about 2% of its blocks have eigenvalues of P^-1 A with negative real
    # part), so what is checked is that the FP32 apply tracks the FP64 apply
    # and that the reported residual is the true one
    runs = {}
    for prec in ("fp64", "fp32"):
        out = ctx.fgmres(b, rd, kp.KP_PC_KSVD, 2, pc, None, prec, restart=30, rtol=1e-10, maxit=300)
        torch.cuda.synchronize()
        r = rd - ctx.operator_apply(b, out["x"])
        true_rel = float(torch.linalg.norm(r) / torch.linalg.norm(rd))
        print(f"  fgmres {prec}: {out['iters']} iterations, relres {out['relres']:.3e}, true {true_rel:.3e}",
              flush=True)
        assert abs(out["relres"] - true_rel) <= 1e-6 * true_rel
        runs[prec] = true_rel
    assert abs(runs["fp32"] / runs["fp64"] - 1.0) <= 0.1


def test_c3_generator_fgmres_converges_at_mesh4(ctx):
    """The 3D p = 7 generator (coupled faces) on a 4^3 periodic mesh, where the
    KSVD preconditioner converges: FP64 and FP32 applies reach 1e-10 (true
    residual), FP32 within one iteration of FP64, and exact block Jacobi
    converges too."""
    import torch

    from paper_1704_04549_amd import kp
    from tests.gpu_util import batch, to_dev
    n, dim, M = 8, 3, 4
    cfg = synth.WORKLOADS["c3_3d_p7"]
    E = M ** dim
    rec = synth.draw_params(E, dim, cfg["seed"], face=True)
    nbr = synth.periodic_neighbours(M, dim)
    synth.mesh_face_velocities(rec, nbr, dim)
    rhs = synth.draw_rhs(E, 1, n ** dim, cfg["rhs_seed"])[:, 0, :]
    b = batch(rec, dim, n, nbr=nbr)
    pc, st = ctx.setup(b, 2)
    rd = to_dev(rhs)
    its = {}
    for prec in ("fp64", "fp32"):
        out = ctx.fgmres(b, rd, kp.KP_PC_KSVD, 2, pc, None, prec, restart=30, rtol=1e-10, maxit=3000)
        torch.cuda.synchronize()
        r = rd - ctx.operator_apply(b, out["x"])
        true_rel = float(torch.linalg.norm(r) / torch.linalg.norm(rd))
        print(f"  mesh 4: fgmres {prec}: {out['iters']} iterations, true relres {true_rel:.2e}", flush=True)
        assert out["converged"] and true_rel <= 1e-10
        its[prec] = out["iters"]
    assert its["fp32"] <= its["fp64"] + 1
    blocks = ctx.build_blocks(b)
    lu, piv, sbj = ctx.blockjacobi_exact(batch(rec, dim, n, blocks=blocks, nbr=nbr))
    out = ctx.fgmres(b, rd, kp.KP_PC_BJ, 2, lu, piv, "fp64", restart=30, rtol=1e-10, maxit=3000)
    torch.cuda.synchronize()
    print(f"  mesh 4: exact block Jacobi {out['iters']} iterations", flush=True)
    assert int(sbj.abs().sum()) == 0 and out["converged"]


def test_c4_fgmres_precisions(ctx):
    """3D p = 15 at full size (4096 elements, block-diagonal, FGMRES(30) to
    1e-10): FP32 and split BF16 applies need at most one iteration more than
    the FP64 apply.  Plain BF16 is outside that bar on this workload (229
    against 226 when measured): it must converge, and its count is printed."""
    from paper_1704_04549_amd import kp
    from tests.gpu_util import batch, to_dev
    w = synth.workload("c4_3d_p15")
    print(f"case c4 fgmres precisions E={w['num_elems']}", flush=True)
    b = batch(w["params"], 3, 16)
    pc, st = ctx.setup(b, 2)
    rd = to_dev(w["rhs"][:, 0, :])
    it = {}
    for prec in ("fp64", "fp32", "bf16x3", "bf16"):
        out = ctx.fgmres(b, rd, pc_kind=kp.KP_PC_KSVD, rank=2, pc_data=pc, pc_prec=prec,
                         restart=30, rtol=1e-10, maxit=3000)
        it[prec] = out["iters"]
        print(f"  {prec}: {out['iters']} iterations, relres {out['relres']:.2e}", flush=True)
        assert out["converged"] and out["relres"] <= 1e-10
    assert it["fp32"] <= it["fp64"] + 1
    assert it["bf16x3"] <= it["fp64"] + 1


def test_c3_block_jacobi_full(ctx):
    """Exact block Jacobi on the whole coupled 3D p = 7 mesh (32768 blocks of
    512 x 512, 64 GiB, factored in place): the solve on sampled elements
    within 1e-12 of the oracle's LU solve of the same blocks.  FGMRES(30) on
    this system stagnates with either preconditioner (exact block Jacobi
    stood at 1.4e-2 after 3000 iterations when measured); with a budget of
    300 iterations the reported residual is the true one, and exact block
    Jacobi ends below the rank-2 KSVD preconditioner.  The factor time and
    both residuals are printed."""
    import torch

    from oracle.krylov import bj_factor, bj_solve
    from paper_1704_04549_amd import kp
    from tests.gpu_util import batch, rel, to_dev
    w = synth.workload("c3_3d_p7")
    n, dim, E = 8, 3, w["num_elems"]
    print(f"case c3 block jacobi E={E}", flush=True)
    b = batch(w["params"], dim, n, nbr=w["nbr"])
    blocks = ctx.build_blocks(b)
    bd = batch(w["params"], dim, n, blocks=blocks, nbr=w["nbr"])
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(ctx.stream)
    lu, piv, st = ctx.blockjacobi_exact(bd, lu=blocks)
    ev1.record(ctx.stream)
    torch.cuda.synchronize()
    t_fact = ev0.elapsed_time(ev1)
    assert int(st.abs().sum()) == 0
    rhs = w["rhs"][:, 0, :]
    rd = to_dev(rhs)
    z = ctx.blockjacobi_solve(bd, lu, piv, rd).cpu().numpy()
    T = tables(n)
    for e in (0, 12345, E - 1):
        A = element_block(w["params"][e], n, dim, T)
        zref = bj_solve(bj_factor(A[None]), rhs[e][None])[0]
        assert rel(z[e], zref) <= 1e-12, e
    res = {}
    pc, _ = ctx.setup(b, 2)
    for name, kw in (("block Jacobi", dict(pc_kind=kp.KP_PC_BJ, pc_data=lu, pc_aux=piv)),
                     ("KSVD fp64", dict(pc_kind=kp.KP_PC_KSVD, pc_data=pc))):
        out = ctx.fgmres(b, rd, rank=2, pc_prec="fp64", restart=30, rtol=1e-10, maxit=300, **kw)
        torch.cuda.synchronize()
        r = rd - ctx.operator_apply(b, out["x"])
        true_rel = float(torch.linalg.norm(r) / torch.linalg.norm(rd))
        print(f"  {name}: {out['iters']} iterations, relres {out['relres']:.3e}, true {true_rel:.3e}", flush=True)
        assert abs(out["relres"] - true_rel) <= 1e-6 * true_rel
        res[name] = true_rel
    print(f"  factor {t_fact:.1f} ms", flush=True)
    assert res["block Jacobi"] < res["KSVD fp64"]
