"""GPU parity of mixed batches (elements of different dimension and degree).

Bars: sigma within 1e-12 of the oracle's SVD; apply against the oracle's
dense solve per element, global relative error <= 1e-12 (FP64), 1e-5 (FP32),
2e-2 (BF16), 1e-4 (split BF16), also after autotuning the launch; the
block-diagonal operator within 1e-13 of || |A| |x| ||; FGMRES on the mixed
system within one iteration of the oracle's FGMRES, FP32 within one of FP64.
"""
import numpy as np
import pytest

import synth
from oracle.apply import dense_solve
from oracle.blocks import element_block
from oracle.krylov import fgmres
from oracle.ksvd import ksvd2d, ksvd3d
from oracle.tables import tables

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1704_04549_amd import kp
    c = kp.Ctx(0)
    yield c
    c.close()


def mixed_case(seed):
    """Classes of (dim, n) with several elements each, shuffled; every element
    closed by its own upwind faces (block-diagonal system)."""
    classes = [(2, 4, 5), (2, 7, 3), (2, 12, 4), (2, 16, 3), (2, 23, 2), (2, 29, 2), (2, 31, 2), (3, 3, 4), (3, 5, 3),
               (3, 8, 3)]
    dims, ns = [], []
    for d, n, k in classes:
        dims += [d] * k
        ns += [n] * k
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(dims))
    dims = np.asarray(dims)[perm]
    ns = np.asarray(ns)[perm]
    recs = np.zeros((len(dims), synth.REC_LEN))
    for e, (d, n) in enumerate(zip(dims, ns)):
        recs[e] = synth.draw_params(1, int(d), seed * 1000 + e, face=True)[0]
    return dims, ns, recs


def oracle_parts(dims, ns, recs):
    blocks, fo = [], []
    for d, n, r in zip(dims, ns, recs):
        A = element_block(r, int(n), int(d), tables(int(n)))
        blocks.append(A)
        fo.append(ksvd2d(A, int(n), 2) if d == 2 else ksvd3d(A, int(n)))
    return blocks, fo


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_mixed_setup_apply_autotune_operator(ctx):
    import torch

    from paper_1704_04549_amd import kp
    from tests.gpu_util import to_dev
    dims, ns, recs = mixed_case(5)
    print(f"mixed E={len(dims)}", flush=True)
    blocks, fo = oracle_parts(dims, ns, recs)
    plan = kp.MixedPlan(ctx, dims, ns, to_dev(recs))
    pc, st = plan.setup()
    _, sg = plan.get_factors(pc)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    sg = sg.cpu().numpy()
    for e, (d, f) in enumerate(zip(dims, fo)):
        so = f["sigma"][:2] if d == 2 else np.r_[f["sigma1"][0], f["sigma2"][:2]]
        got = sg[e, :2] if d == 2 else sg[e, :3]
        assert np.max(np.abs(got / so - 1)) <= 1e-12, e
    off = plan.offsets
    r = np.random.default_rng(1).standard_normal(plan.vec_len)
    zref = np.concatenate([dense_solve(fo[e], r[off[e]:off[e + 1]]) for e in range(len(dims))])
    rd = to_dev(r)
    outs = {}
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5), ("bf16", 2e-2), ("bf16x3", 1e-4)):
        z = plan.apply(pc, prec, rd).cpu().numpy()
        outs[prec] = z
        print(f"  {prec}: {rel(z, zref):.2e}", flush=True)
        assert rel(z, zref) <= tol, prec
    # autotuned launch: the same per-element arithmetic (the workgroup and the
    # wave paths are separate instantiations, so FP32 rounding may differ in
    # the last bit); the oracle bars hold after tuning
    scratch = torch.empty_like(rd)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        modes = plan.autotune(pc, prec, rd, scratch)
        print(f"  autotune {prec}: {modes}", flush=True)
        assert set(modes) == set(zip(dims.tolist(), ns.tolist()))
        z = plan.apply(pc, prec, rd).cpu().numpy()
        assert rel(z, zref) <= tol
        assert rel(z, outs[prec]) <= 10 * np.finfo(np.float64 if prec == "fp64" else np.float32).eps
    # block-diagonal operator
    x = np.random.default_rng(2).standard_normal(plan.vec_len)
    y = plan.operator_apply(to_dev(x)).cpu().numpy()
    yref = np.concatenate([blocks[e] @ x[off[e]:off[e + 1]] for e in range(len(dims))])
    # forward error of a product: relative to || |A| |x| || (the n = 31 blocks cancel heavily)
    yabs = np.concatenate([np.abs(blocks[e]) @ np.abs(x[off[e]:off[e + 1]]) for e in range(len(dims))])
    assert np.linalg.norm(y - yref) <= 1e-13 * np.linalg.norm(yabs)
    plan.close()


def test_mixed_autotune_large_3d(ctx):
    """3D n = 12 and 16 elements: four of them per workgroup would not fit in
    LDS at FP64, so the autotuner keeps those classes on whole workgroups; the
    list tuned at FP32 then serves every precision."""
    import torch

    from paper_1704_04549_amd import kp
    from tests.gpu_util import to_dev
    dims = np.array([3, 2, 3, 3, 2, 3])
    ns = np.array([16, 31, 12, 4, 9, 16])
    recs = np.zeros((len(dims), synth.REC_LEN))
    for e, (d, n) in enumerate(zip(dims, ns)):
        recs[e] = synth.draw_params(1, int(d), 7000 + e, face=True)[0]
    print(f"mixed large E={len(dims)}", flush=True)
    _, fo = oracle_parts(dims, ns, recs)
    plan = kp.MixedPlan(ctx, dims, ns, to_dev(recs))
    pc, st = plan.setup()
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    off = plan.offsets
    r = np.random.default_rng(4).standard_normal(plan.vec_len)
    zref = np.concatenate([dense_solve(fo[e], r[off[e]:off[e + 1]]) for e in range(len(dims))])
    rd = to_dev(r)
    modes = plan.autotune(pc, "fp32", rd, torch.empty_like(rd))
    print(f"  modes {modes}", flush=True)
    assert modes[(3, 16)] == 0 and modes[(3, 12)] == 0
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5), ("bf16", 2e-2), ("bf16x3", 1e-4)):
        z = plan.apply(pc, prec, rd).cpu().numpy()
        print(f"  {prec}: {rel(z, zref):.2e}", flush=True)
        assert rel(z, zref) <= tol, prec
    plan.close()


def test_mixed_fgmres_matches_oracle(ctx):
    from paper_1704_04549_amd import kp
    from tests.gpu_util import to_dev
    dims, ns, recs = mixed_case(9)
    blocks, fo = oracle_parts(dims, ns, recs)
    plan = kp.MixedPlan(ctx, dims, ns, to_dev(recs))
    pc, _ = plan.setup()
    off = plan.offsets
    E = len(dims)
    b = np.random.default_rng(3).standard_normal(plan.vec_len)
    Aop = lambda v: np.concatenate([blocks[e] @ v[off[e]:off[e + 1]] for e in range(E)])
    import scipy.linalg as sla
    from oracle.ksvd import precond_matrix
    lus = [sla.lu_factor(precond_matrix(f)) for f in fo]
    Mop = lambda v: np.concatenate([sla.lu_solve(lus[e], v[off[e]:off[e + 1]]) for e in range(E)])
    print("  oracle FGMRES ...", flush=True)
    _, it_ref, _, ok = fgmres(Aop, Mop, b, m=30, rtol=1e-10, maxit=400)
    assert ok
    xref = np.concatenate([np.linalg.solve(blocks[e], b[off[e]:off[e + 1]]) for e in range(E)])
    res = {}
    for prec in ("fp64", "fp32"):
        out = plan.fgmres(to_dev(b), pc_kind=kp.KP_PC_KSVD, precond=pc, pc_prec=prec)
        res[prec] = out["iters"]
        print(f"  {prec}: iters {out['iters']} (oracle {it_ref})", flush=True)
        assert out["converged"]
        assert rel(out["x"].cpu().numpy(), xref) <= 1e-8
    assert abs(res["fp64"] - it_ref) <= 1
    assert res["fp32"] <= res["fp64"] + 1
    plan.close()


def test_mixed_setup_concurrent_classes_deterministic(ctx):
    """The table kernels of the (dim, n) classes run concurrently on the plan's
    side streams and are joined back to the context's stream: a setup read
    right after it on the context's stream (no device-wide sync) holds exactly
    the bytes of a setup read after a full synchronisation, and repeated
    setups agree bit for bit."""
    import torch

    from paper_1704_04549_amd import kp
    from tests.gpu_util import to_dev
    dims, ns, recs = mixed_case(11)
    print(f"mixed E={len(dims)} classes={len(set(zip(dims.tolist(), ns.tolist())))}", flush=True)
    plan = kp.MixedPlan(ctx, dims, ns, to_dev(recs))
    dev = ctx.device
    ref = torch.zeros(plan.precond_bytes, dtype=torch.uint8, device=dev)
    st = torch.empty(plan.E, dtype=torch.int32, device=dev)
    plan.setup(ref, st)
    torch.cuda.synchronize()
    ref_h = ref.cpu()
    assert int(st.abs().sum()) == 0
    for rep in range(3):
        buf = torch.zeros(plan.precond_bytes, dtype=torch.uint8, device=dev)
        plan.setup(buf, st)
        got = buf.to("cpu")  # ordered on the context's stream only
        assert torch.equal(got, ref_h), rep
    plan.close()
