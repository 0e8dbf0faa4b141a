"""GPU parity of the 2D rank-3 preconditioner (three Kronecker terms).

The paper inverts two-term sums directly (Sec. 4.2); with a third term the
library solves P3 z = r per element by flexible GMRES preconditioned with the
rank-2 apply.  Bars:
  * setup: sigma_1..3 relative <= 1e-12, P3 from GPU factors vs oracle <= 1e-12;
  * apply on the oracle's factors, against the dense solve of the oracle's P3:
    global relative <= 1e-12 (FP64), <= 1e-5 (FP32), <= 2e-2 (BF16), <= 1e-4
    (split BF16);
  * setup + apply end to end (FP64): global <= 1e-12, and every element within
    max(1e-12, 100 kappa(P3) eps).
"""
import numpy as np
import pytest

import synth
from oracle.apply import dense_solve
from oracle.blocks import element_block
from oracle.ksvd import factor_array, factors_from_array, ksvd2d, precond_matrix
from oracle.tables import tables

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def ctx():
    from paper_1704_04549_amd import kp
    c = kp.Ctx(0)
    yield c
    c.close()


CASES = [  # n, elements, rhs per element, explicit blocks
    (16, 24, 3, False),
    (16, 9, 2, True),
    (8, 40, 2, True),
    (5, 17, 1, False),
]


@pytest.mark.parametrize("n,E,nrhs,explicit", CASES)
def test_rank3_setup_and_apply(ctx, n, E, nrhs, explicit):
    import torch

    from tests.gpu_util import batch, rel, to_dev
    print(f"rank3 n={n} E={E} nrhs={nrhs} explicit={explicit}", flush=True)
    params = synth.draw_params(E, 2, 1002)
    T = tables(n)
    blocks = np.stack([element_block(r, n, 2, T) for r in params])
    fo = [ksvd2d(A, n, 3) for A in blocks]
    b = batch(params, 2, n, blocks=blocks if explicit else None)
    pc, st = ctx.setup(b, 3)
    f_gpu, s_gpu = ctx.get_factors(b, 3, pc)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0, st.cpu().numpy()
    f_gpu = f_gpu.cpu().numpy()
    s_gpu = s_gpu.cpu().numpy()
    for e in range(E):
        assert np.max(np.abs(s_gpu[e, :3] / fo[e]["sigma"][:3] - 1)) <= 1e-12, e
        assert rel(precond_matrix(factors_from_array(f_gpu[e], 2)), precond_matrix(fo[e])) <= 1e-12, e
    r = np.random.default_rng(n + E).standard_normal((E, nrhs, n * n))
    zref = np.stack([dense_solve(fo[e], r[e]) for e in range(E)])
    rd = to_dev(r)
    # end to end (GPU setup), FP64
    z = ctx.apply(b, 3, pc, "fp64", rd).cpu().numpy()
    assert rel(z, zref) <= 1e-12
    for e in range(E):
        kap = np.linalg.cond(precond_matrix(fo[e]))
        assert rel(z[e], zref[e]) <= max(1e-12, 100 * kap * EPS), e
    # every precision on the oracle's factors
    Fo = to_dev(np.stack([factor_array(f) for f in fo]))
    pco, sto = ctx.setup_from_factors(b, 3, Fo)
    torch.cuda.synchronize()
    assert int(sto.abs().sum()) == 0
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5), ("bf16", 2e-2), ("bf16x3", 1e-4)):
        zp = ctx.apply(b, 3, pco, prec, rd).cpu().numpy()
        err = rel(zp, zref)
        print(f"  {prec}: {err:.2e}", flush=True)
        assert err <= tol, (prec, err)


def test_rank3_zero_rhs_gives_zero(ctx):
    import torch

    from tests.gpu_util import batch, to_dev
    n, E = 6, 5
    params = synth.draw_params(E, 2, 9)
    b = batch(params, 2, n)
    pc, _ = ctx.setup(b, 3)
    z = ctx.apply(b, 3, pc, "fp64", to_dev(np.zeros((E, n * n))))
    torch.cuda.synchronize()
    assert not z.cpu().numpy().any()


def test_rank3_n16_series_path_matches_oracle_and_gmres_path(ctx):
    """n = 16: the matrix-core Neumann series over the rank-2 apply (16
    right-hand sides per workgroup; 18 here, so two ragged groups) against the
    dense solve of the oracle's P3 at every precision's bar, and against the
    per-element GMRES path (KP_OPT_APPLY_MFMA16 = 0) to the same bars."""
    import torch

    from paper_1704_04549_amd import kp
    from tests.gpu_util import batch, rel, to_dev
    n, E, nrhs = 16, 12, 18
    print(f"rank3 series n={n} E={E} nrhs={nrhs}", flush=True)
    params = synth.draw_params(E, 2, 1202)
    T = tables(n)
    blocks = np.stack([element_block(r, n, 2, T) for r in params])
    fo = [ksvd2d(A, n, 3) for A in blocks]
    b = batch(params, 2, n)
    Fo = to_dev(np.stack([factor_array(f) for f in fo]))
    pco, sto = ctx.setup_from_factors(b, 3, Fo)
    torch.cuda.synchronize()
    assert int(sto.abs().sum()) == 0
    r = np.random.default_rng(77).standard_normal((E, nrhs, n * n))
    zref = np.stack([dense_solve(fo[e], r[e]) for e in range(E)])
    rd = to_dev(r)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5), ("bf16", 2e-2), ("bf16x3", 1e-4)):
        zs = ctx.apply(b, 3, pco, prec, rd).cpu().numpy()
        ctx.set_option(kp.KP_OPT_APPLY_MFMA16, 0)
        zg = ctx.apply(b, 3, pco, prec, rd).cpu().numpy()
        ctx.set_option(kp.KP_OPT_APPLY_MFMA16, 1)
        print(f"  {prec}: series {rel(zs, zref):.2e} gmres {rel(zg, zref):.2e}", flush=True)
        assert rel(zs, zref) <= tol and rel(zg, zref) <= tol


def test_rank3_n16_divergent_series_falls_back(ctx):
    """A third term large enough that the Neumann series diverges
    (A3 = 3 A1, B3 = B1): every element is flagged and solved by the
    per-element GMRES; FP64 and FP32 against the dense solve of that P3."""
    import torch

    from tests.gpu_util import batch, rel, to_dev
    n, E, nrhs = 16, 5, 2
    params = synth.draw_params(E, 2, 1303)
    T = tables(n)
    blocks = np.stack([element_block(r, n, 2, T) for r in params])
    fo = []
    for A in blocks:
        f = ksvd2d(A, n, 2)
        f = dict(f, rank=3, A=[f["A"][0], f["A"][1], 3.0 * f["A"][0]], B=[f["B"][0], f["B"][1], f["B"][0]])
        fo.append(f)
    b = batch(params, 2, n)
    pco, sto = ctx.setup_from_factors(b, 3, to_dev(np.stack([factor_array(f) for f in fo])))
    torch.cuda.synchronize()
    assert int(sto.abs().sum()) == 0
    r = np.random.default_rng(5).standard_normal((E, nrhs, n * n))
    zref = np.stack([dense_solve(fo[e], r[e]) for e in range(E)])
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        z = ctx.apply(b, 3, pco, prec, to_dev(r)).cpu().numpy()
        print(f"  divergent series {prec}: {rel(z, zref):.2e}", flush=True)
        assert rel(z, zref) <= tol
