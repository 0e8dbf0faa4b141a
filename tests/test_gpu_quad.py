"""General elements (non-collocated quadrature, per-point coefficients):
kp_setup_quad against the oracle.

Bars: sigma within 1e-12 and P within 1e-12 (relative) of the oracle's full
SVD of the block assembled by its quadrature definition (oracle/shuffled.py);
z = P^{-1} r within 1e-12 (FP64), 1e-5 (FP32), 1e-4 (split BF16), 2e-2 (BF16)
globally, on ragged batch sizes in 2D and 3D; at n = 16, mu = 17 in 3D
(256 elements) the same bars on three elements against stored oracle
results (tests/golden/quad_sampled.npz, written by
tests/golden/make_quad_sampled.py from oracle/ alone), every element's
status zero, and the setup time printed.
"""
import os

import numpy as np
import pytest

import synth
from oracle import shuffled
from oracle.apply import dense_solve
from oracle.ksvd import factors_from_array, ksvd2d, ksvd3d, precond_matrix

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-4, "bf16": 2e-2}


@pytest.fixture(scope="module")
def ctx():
    from paper_1704_04549_amd import kp
    c = kp.Ctx(0)
    yield c
    c.close()


def quad_batch(q, n):
    from paper_1704_04549_amd import kp
    from tests.gpu_util import to_dev
    return kp.QuadBatch(q["dim"], n, q["mu"], q["tau"], to_dev(q["c"]), to_dev(q["a"]), to_dev(q["nu"]),
                        to_dev(q["g"]))


@pytest.mark.parametrize("dim,n,mu,E", [(2, 5, 7, 13), (2, 16, 17, 9), (3, 4, 6, 37), (3, 8, 9, 7),
                                        (3, 8, 12, 5)])
def test_quad_setup_and_apply_match_oracle(ctx, dim, n, mu, E):
    import torch

    from tests.gpu_util import rel, to_dev
    print(f"quad dim={dim} n={n} mu={mu} E={E}", flush=True)
    q = synth.quad_elements(E, dim, mu, seed=300 + n + mu)
    qb = quad_batch(q, n)
    pc, st = ctx.setup_quad(qb)
    b = qb.batch()
    F, sig = ctx.get_factors(b, 2, pc)
    r = np.random.default_rng(n + mu).standard_normal((E, n ** dim))
    zs = {p: ctx.apply(b, 2, pc, p, to_dev(r)).cpu().numpy() for p in TOL}
    torch.cuda.synchronize()
    assert int((st != 0).sum()) == 0
    F, sig = F.cpu().numpy(), sig.cpu().numpy()
    Q = shuffled.quad_tables(n, mu)
    zref = []
    for e in range(E):
        A = shuffled.element_block(synth.quad_element(q, e, n), Q)
        f = ksvd2d(A, n, 2) if dim == 2 else ksvd3d(A, n)
        so = f["sigma"][:2] if dim == 2 else np.r_[f["sigma1"][0], f["sigma2"][:2]]
        assert np.max(np.abs(sig[e, :len(so)] / so - 1)) <= 1e-12, e
        Pg = precond_matrix(factors_from_array(F[e], dim))
        Po = precond_matrix(f)
        assert np.linalg.norm(Pg - Po) <= 1e-12 * np.linalg.norm(Po), e
        zref.append(dense_solve(f, r[e]))
    zref = np.array(zref)
    for p, tol in TOL.items():
        err = rel(zs[p], zref)
        print(f"  {p}: {err:.2e}", flush=True)
        assert err <= tol, (p, err)


def test_quad_3d_p15_sampled(ctx):
    import torch

    from tests.gpu_util import rel, to_dev
    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "quad_sampled.npz"))
    n, mu, E = int(g["n"]), int(g["mu"]), int(g["num_elems"])
    print(f"quad 3d n={n} mu={mu} E={E}", flush=True)
    q = synth.quad_elements(E, 3, mu)
    qb = quad_batch(q, n)
    pc, st = ctx.setup_quad(qb)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(ctx.stream)
    ctx.setup_quad(qb, precond=pc, status=st)
    ev1.record(ctx.stream)
    torch.cuda.synchronize()
    print(f"  setup {ev0.elapsed_time(ev1):.2f} ms for {E} elements", flush=True)
    b = qb.batch()
    _, sig = ctx.get_factors(b, 2, pc)
    sig = sig.cpu().numpy()
    assert int((st != 0).sum()) == 0
    idx = g["idx"]
    assert np.max(np.abs(sig[idx, :3] / g["sigma"] - 1)) <= 1e-12
    r = np.random.default_rng(int(g["rhs_seed"])).standard_normal((E, n ** 3))
    for p, tol in TOL.items():
        z = ctx.apply(b, 2, pc, p, to_dev(r)).cpu().numpy()
        err = rel(z[idx], g["z"])
        print(f"  {p}: {err:.2e}", flush=True)
        assert err <= tol, (p, err)
