"""Benchmark: preconditioner setup + apply throughput at equal FGMRES iterations.

Workload (default): 3D, p = 15 (n = 16), 4096 elements (a 16^3 hex mesh's
worth), synthetic records from the seeded generator, each element closed by
its own upwind faces (block-diagonal global system), rank-2 two-stage KSVD,
matrix-free setup, FP32 apply inside an FP64 FGMRES(30) to 1e-10.

One step = one whole pass of the hot path over the batch: kp_setup (Lanczos
KSVD of every element, factor inversion, Schur forms, apply tables) followed by
N applies of the preconditioner to one right-hand side per element, where N is
the FGMRES iteration count the same preconditioner needed (measured before the
timed region, together with the plain FP64 preconditioner's count; the
variant is valid only if N <= N_fp64 + 1).
value = DOF * N / (time per step): setup + apply DOF/s of the whole batch.

Also reported: the plain FP64 preconditioner's rate on the same workload
(speedup_vs_fp64), the roofline of the dominant kernel measured with HIP
events on the library's stream, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "precond setup+apply DOF/s vs plain FP64 at equal FGMRES iterations, 3D p=15"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c4_3d_p15")
    ap.add_argument("--prec", default="fp32", choices=["fp32", "bf16", "bf16x3", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=3)
    return ap.parse_args()


def cpu_baseline(w, n, dim, N_iter, sample):
    """The oracle on `sample` elements: full-SVD KSVD + dense LU of P (setup), LU solves (apply)."""
    import scipy.linalg as sla
    from threadpoolctl import threadpool_info

    from oracle.blocks import element_block
    from oracle.ksvd import ksvd2d, ksvd3d, precond_matrix
    from oracle.tables import tables

    T = tables(n)
    idx = np.linspace(0, w["num_elems"] - 1, sample).astype(int)
    t_setup = 0.0
    t_apply = 0.0
    for e in idx:
        t0 = time.perf_counter()
        A = element_block(w["params"][e], n, dim, T)
        f = ksvd3d(A, n) if dim == 3 else ksvd2d(A, n, 2)
        lu = sla.lu_factor(precond_matrix(f))
        t1 = time.perf_counter()
        sla.lu_solve(lu, w["rhs"][e, 0])
        t2 = time.perf_counter()
        t_setup += t1 - t0
        t_apply += t2 - t1
    dof = sample * n ** dim
    value = dof * N_iter / (t_setup + N_iter * t_apply)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return dict(value=value, unit="DOF/s", cores=int(threads), kind="oracle",
                sample=f"{sample} elements (indices {idx.tolist()}), setup {t_setup:.2f}s, "
                       f"one apply {t_apply:.3f}s, N={N_iter}")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import synth
    from paper_1704_04549_amd import kp

    w = synth.workload(args.workload)
    dim, n, E = w["dim"], w["n"], w["num_elems"]
    dev = torch.device("cuda", 0)
    params = torch.from_numpy(w["params"]).to(dev)
    nbr = torch.from_numpy(w["nbr"]).to(dev) if w["nbr"] is not None else None
    rhs = torch.from_numpy(np.ascontiguousarray(w["rhs"][:, 0, :])).to(dev)
    ctx = kp.Ctx(0)
    b = kp.Batch(params, dim, n, nbr=nbr)
    rank = w["rank"]
    ndof = E * n ** dim
    pc, st = ctx.setup(b, rank)
    z = torch.empty_like(rhs)
    # iteration counts (outside the timed region)
    out64 = ctx.fgmres(b, rhs, pc_kind=kp.KP_PC_KSVD, rank=rank, pc_data=pc, pc_prec="fp64",
                       restart=30, rtol=1e-10, maxit=3000)
    outv = ctx.fgmres(b, rhs, pc_kind=kp.KP_PC_KSVD, rank=rank, pc_data=pc, pc_prec=args.prec,
                      restart=30, rtol=1e-10, maxit=3000)
    n64, nv = out64["iters"], outv["iters"]
    valid = outv["converged"] and out64["converged"] and nv <= n64 + 1

    def step(prec, N):
        ctx.setup(b, rank, precond=pc, status=st)
        for _ in range(N):
            ctx.apply(b, rank, pc, prec, rhs, z)

    def timed(prec, N, K, W):
        for _ in range(W):
            step(prec, N)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            step(prec, N)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / K

    sec = timed(args.prec, nv, args.steps, args.warmup)
    sec64 = timed("fp64", n64, max(3, args.steps // 4), 1)
    value = ndof * nv / sec
    value64 = ndof * n64 / sec64

    # per-kernel durations with HIP events on the library's stream
    def event_ms(fn, reps):
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        fn()
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / reps

    t_apply = event_ms(lambda: ctx.apply(b, rank, pc, args.prec, rhs, z), 20)
    t_setup = event_ms(lambda: ctx.setup(b, rank, precond=pc, status=st), 5)
    tab_bytes = {"fp64": 8, "fp32": 4, "bf16": 2, "bf16x3": 4}[args.prec]
    ne = (7 + n) * n * n
    apply_bytes = ndof * 16 + E * ne * tab_bytes
    apply_share = nv * t_apply / (nv * t_apply + t_setup)
    if apply_share >= 0.5:
        achieved = apply_bytes / (t_apply * 1e-3) / 1e9
        roof = {"kernel": "apply", "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "ms_per_launch": round(t_apply, 4),
                "algorithmic_bytes": int(apply_bytes)}
    else:
        # setup is a chain of latency-bound per-element solves; report its rate
        rec_bytes = E * 12 * 8 + E * (4 + 5 * n * n + ne * 20)
        achieved = rec_bytes / (t_setup * 1e-3) / 1e9
        roof = {"kernel": "setup", "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "ms_per_launch": round(t_setup, 4),
                "algorithmic_bytes": int(rec_bytes)}
    line = {
        "metric": METRIC,
        "value": value if valid else None,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": f"3D p={n - 1} (n={n}), {E} elements, upwind-closed element "
                               f"blocks (block-diagonal system), rank 2 two-stage KSVD, "
                               f"matrix-free setup, {args.prec} apply, FP64 FGMRES(30) to 1e-10",
                   "elements": E, "dof": ndof, "precision": args.prec,
                   "fgmres_iters": nv, "fgmres_iters_fp64": n64, "valid": valid},
        "fp64_value": value64,
        "speedup_vs_fp64": value / value64 if valid else None,
        "setup_ms": t_setup,
        "apply_ms": t_apply,
        "setup_dof_per_s": ndof / (t_setup * 1e-3),
        "apply_dof_per_s": ndof / (t_apply * 1e-3),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, n, dim, nv, args.cpu_sample)
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
