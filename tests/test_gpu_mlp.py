"""GPU parity of the learned setup against the FP64 oracle (oracle/mlp.py).

Bars:
  * network outputs and the loss gradient with FP32 matrix-core GEMMs within
    1e-5 (relative, global) of the FP64 oracle on the same FP32 parameters;
    bf16 GEMMs within 2e-2;
  * predictions from records (features, normalisation, network, block
    scales) within 1e-5 of the oracle;
  * training lowers the loss at least tenfold;
  * the acceptance decisions equal the host evaluation of the same
    closed-form criterion on the same predicted factors (elements within
    1e-9 of the threshold excepted), and the accepted factors' apply matches
    the oracle's dense solve of the predicted P within 1e-12;
  * rejected elements and the warm-start mode reproduce the SVD setup
    (sigma within 1e-12, apply within 1e-12);
  * the gain: a trained network is accepted on most validation elements,
    an untrained one on none.
"""
import ctypes
import os

import numpy as np
import pytest

import synth
from oracle import mlp as omlp
from oracle.apply import dense_solve
from oracle.ksvd import factors_from_array

pytestmark = pytest.mark.gpu

HOSTLIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_native", "libkp_hostcheck.so")


@pytest.fixture(scope="module")
def ctx():
    from paper_1704_04549_amd import kp
    c = kp.Ctx(0)
    yield c
    c.close()


def kaiming(I, H, O, seed, out_scale=0.1):
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((H, I)) * np.sqrt(2.0 / I)
    W2 = rng.standard_normal((H, H)) * np.sqrt(2.0 / H)
    W3 = rng.standard_normal((O, H)) * np.sqrt(2.0 / H) * out_scale
    b1 = rng.standard_normal(H) * 0.1
    b2 = rng.standard_normal(H) * 0.1
    b3 = rng.standard_normal(O) * 0.01
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3]).astype(np.float32)


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dim,n,H,N", [(3, 3, 37, 50), (2, 4, 64, 70)])
def test_forward_and_gradient_match_oracle(ctx, dim, n, H, N):
    from tests.gpu_util import to_dev
    print(f"mlp grad dim={dim} n={n} H={H} N={N}", flush=True)
    I, O = 12, omlp.n_outputs(dim, n)
    p32 = kaiming(I, H, O, 11, out_scale=1.0)
    model = ctx.mlp_create(dim, n, H, to_dev(p32))
    rng = np.random.default_rng(12)
    x = rng.standard_normal((N, I)).astype(np.float32)
    p64 = p32.astype(np.float64)
    y_ref, _ = omlp.forward(p64, x.astype(np.float64), I, H, O)
    # targets: the outputs under a random P-preserving sign pattern per row, plus
    # noise of the outputs' own size, so that every row's sign choice is
    # exercised away from a tie and the residual y - s t (which drives the
    # gradient) is not a small difference of large numbers
    S = omlp.block_signs(dim, n)
    t = (S[rng.integers(0, S.shape[0], N)] * y_ref +
         1.0 * np.std(y_ref) * rng.standard_normal((N, O))).astype(np.float32)
    loss_ref, g_ref = omlp.loss_and_grad(p64, x.astype(np.float64), t.astype(np.float64), I, H, O, dim, n)
    _, _, _, costs = omlp.loss_and_grad_y(y_ref, t.astype(np.float64), dim, n)
    srt = np.sort(costs, axis=1)
    assert np.all(srt[:, 1] - srt[:, 0] > 0.03 * srt[:, 0])
    for prec, tol in (("fp32", 1e-5), ("bf16", 2e-2)):
        y = ctx.mlp_forward(model, to_dev(x), O, prec).cpu().numpy()
        assert rel(y, y_ref) <= tol, (prec, rel(y, y_ref))
        loss, g = ctx.mlp_loss_grad(model, to_dev(x), to_dev(t), p32.size, prec)
        loss = float(loss.cpu().numpy()[0])
        g = g.cpu().numpy()
        print(f"  {prec}: y {rel(y, y_ref):.2e} loss {abs(loss - loss_ref) / loss_ref:.2e} grad {rel(g, g_ref):.2e}",
              flush=True)
        assert abs(loss - loss_ref) <= tol * loss_ref
        assert rel(g, g_ref) <= tol, (prec, rel(g, g_ref))


def train_model(ctx, dim, n, H, E, epochs, prec="fp32"):
    from paper_1704_04549_amd import kp
    from tests.gpu_util import batch, to_dev
    tr = synth.draw_params(E, dim, synth.MLP_TRAIN_SEED, face=(dim == 3))
    btr = batch(tr, dim, n)
    pc, st = ctx.setup(btr, 2)
    F, _ = ctx.get_factors(btr, 2, pc)
    O = omlp.n_outputs(dim, n)
    model = ctx.mlp_create(dim, n, H, to_dev(kaiming(12, H, O, 5004)))
    hist = ctx.mlp_train(model, btr, F, epochs=epochs, batch=256, lr=1e-3, seed=synth.MLP_TRAIN_SEED, prec=prec)
    return model, hist, kp


@pytest.mark.parametrize("dim,n", [(3, 8), (2, 8)])
def test_train_predict_and_learned_setup(ctx, dim, n):
    import torch

    from tests.gpu_util import batch, to_dev
    print(f"mlp train dim={dim} n={n}", flush=True)
    H = 128
    model, hist, kp = train_model(ctx, dim, n, H, 4000, 30)
    print(f"  loss {hist[0]:.4f} -> {hist[-1]:.5f}", flush=True)
    assert hist[-1] <= 0.1 * hist[0]
    va = synth.draw_params(400, dim, synth.MLP_VAL_SEED, face=(dim == 3))
    bva = batch(va, dim, n)
    # predictions from records against the oracle with the model's own normalisation
    params, xm, xs, ys = (t.cpu().numpy().astype(np.float64) for t in ctx.mlp_get(model, dim, n, H))
    O = omlp.n_outputs(dim, n)
    xn = (omlp.features(va, dim) - xm) / xs
    y_ref, _ = omlp.forward(params, xn, 12, H, O)
    F_ref = y_ref * np.repeat(ys, n * n)[None, :]
    F_gpu = ctx.mlp_predict(model, bva).cpu().numpy().reshape(len(va), -1)
    assert rel(F_gpu, F_ref) <= 1e-5
    # learned setup
    ctx.set_model(model)
    pcL, stL = ctx.setup(bva, 2, mode=kp.KP_SETUP_LEARNED)
    pcS, stS = ctx.setup(bva, 2)
    torch.cuda.synchronize()
    stL = stL.cpu().numpy()
    assert not stS.cpu().numpy().any()
    acc = stL == 0
    print(f"  accepted {acc.sum()} of {len(va)}; statuses {np.unique(stL).tolist()}", flush=True)
    assert set(np.unique(stL).tolist()) <= {0, 48}
    # decisions against the host evaluation of the criterion on the same factors
    lib = ctypes.CDLL(HOSTLIB)
    lib.kph_learned_check.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_double, ctypes.c_void_p]
    Fp = ctx.mlp_predict(model, bva).cpu().numpy()
    out = np.zeros(8)
    for e in range(len(va)):
        f = np.ascontiguousarray(Fp[e])
        ok = lib.kph_learned_check(dim, n, va[e].ctypes.data_as(ctypes.c_void_p),
                                   f.ctypes.data_as(ctypes.c_void_p), 1.1, out.ctypes.data_as(ctypes.c_void_p))
        margin = min(abs(out[0] - 1.1 * out[1] - 1e-12 * out[2]), abs(out[0] - out[2])) / out[2]
        if margin > 1e-9:
            assert ok == int(acc[e]), e
    # accepted: the apply inverts the predicted P; rejected: the SVD's factors
    fL, sL = ctx.get_factors(bva, 2, pcL)
    fS, sS = ctx.get_factors(bva, 2, pcS)
    fL, sL, fS, sS = (t.cpu().numpy() for t in (fL, sL, fS, sS))
    nsig = 3 if dim == 3 else 2
    rej = np.where(~acc)[0]
    if rej.size:
        assert np.max(np.abs(sL[rej, :nsig] / sS[rej, :nsig] - 1)) <= 1e-12
    r = np.random.default_rng(3).standard_normal((len(va), n ** dim))
    zL = ctx.apply(bva, 2, pcL, "fp64", to_dev(r)).cpu().numpy()
    zS = ctx.apply(bva, 2, pcS, "fp64", to_dev(r)).cpu().numpy()
    if rej.size:
        assert rel(zL[rej], zS[rej]) <= 1e-12
    for e in np.where(acc)[0][:3]:
        zref = dense_solve(factors_from_array(Fp[e], dim), r[e])
        assert rel(zL[e], zref) <= 1e-12, e
    # the gain over the method without a network: an untrained (zero) model is never accepted
    zero = ctx.mlp_create(dim, n, H, None)
    ctx.set_model(zero)
    _, st0 = ctx.setup(bva, 2, mode=kp.KP_SETUP_LEARNED)
    st0 = st0.cpu().numpy()
    print(f"  untrained accepted {(st0 == 0).sum()}", flush=True)
    assert (st0 == 0).sum() == 0
    if dim == 3:
        # the 3D two-stage KSVD leaves ~20-35% of ||A||, so a prediction a few
        # per cent off can be within 1.1x of it; the 2D KSVD leaves ~1%, which
        # this network does not approach: there every element falls back to
        # the warm-started Lanczos (checked above)
        assert acc.mean() >= 0.2
    ctx.set_model(None)


def test_c4_recipe_acceptance_and_setup_time(ctx):
    """The 3D p = 15 recipe: 20000 training elements (seed 3004), 2000
    validation elements (seed 4004), H = 256, 60 epochs.  The trained network
    is accepted on most validation elements; accepted elements keep the
    closed-form criterion.  Both setup times are reported: since the SVD
    setup forms the mass tensor's Gram products once per element, the two
    take about the same time, so no order between them is asserted."""
    import torch

    from tests.gpu_util import batch
    dim, n = 3, 16
    model, hist, kp = train_model(ctx, dim, n, 256, 20000, 60)
    print(f"  loss {hist[0]:.4f} -> {hist[-1]:.5f}", flush=True)
    assert hist[-1] <= 0.05 * hist[0]
    va = synth.draw_params(2000, dim, synth.MLP_VAL_SEED, face=True)
    b = batch(va, dim, n)
    ctx.set_model(model)

    def timed(mode):
        pc, st = ctx.setup(b, 2, mode=mode)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(3):
            ctx.setup(b, 2, mode=mode, precond=pc, status=st)
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / 3, st.cpu().numpy()

    t_svd, _ = timed(kp.KP_SETUP_SVD)
    t_l, st = timed(kp.KP_SETUP_LEARNED)
    frac = float((st == 0).mean())
    print(f"  accepted {frac:.3f}; setup ms: svd {t_svd:.2f} learned {t_l:.2f}", flush=True)
    assert frac >= 0.7
    assert t_l > 0.0 and t_svd > 0.0
    ctx.set_model(None)


def test_warm_mode_reproduces_svd_setup(ctx):
    import torch

    from tests.gpu_util import batch, to_dev
    dim, n = 3, 8
    model, hist, kp = train_model(ctx, dim, n, 64, 1500, 10, prec="bf16")
    assert hist[-1] < hist[0]
    w = synth.draw_params(300, dim, 77, face=True)
    b = batch(w, dim, n)
    ctx.set_model(model)
    pcW, stW = ctx.setup(b, 2, mode=kp.KP_SETUP_LEARNED_WARM)
    pcS, _ = ctx.setup(b, 2)
    torch.cuda.synchronize()
    assert set(np.unique(stW.cpu().numpy()).tolist()) <= {0, 32}
    _, sW = ctx.get_factors(b, 2, pcW)
    _, sS = ctx.get_factors(b, 2, pcS)
    assert float(((sW[:, :3] / sS[:, :3]) - 1).abs().max()) <= 1e-12
    r = to_dev(np.random.default_rng(4).standard_normal((300, n ** dim)))
    zW = ctx.apply(b, 2, pcW, "fp64", r).cpu().numpy()
    zS = ctx.apply(b, 2, pcS, "fp64", r).cpu().numpy()
    assert rel(zW, zS) <= 1e-12
    ctx.set_model(None)
