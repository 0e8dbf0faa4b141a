"""CPU checks of the GPU library's per-element arithmetic (host build of elem_ops.h).

The same source the kernels run, built for the host with a one-thread team,
is checked here against the oracle without a GPU: 1D tables, element blocks,
the Lanczos KSVD setup (explicit and matrix-free), the device real Schur form,
table formation and the apply in every precision.
"""
import ctypes
import os

import numpy as np
import pytest

import synth
from oracle.apply import dense_solve
from oracle.blocks import element_block
from oracle.ksvd import factor_array, factors_from_array, ksvd2d, ksvd3d, precond_matrix
from oracle.tables import tables

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_native", "libkp_hostcheck.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="host-check build missing (run build)")


def P(a):
    return a.ctypes.data_as(ctypes.c_void_p)


@pytest.fixture(scope="module")
def lib():
    return ctypes.CDLL(LIB)


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


@pytest.mark.parametrize("n", [2, 5, 8, 16, 31])
def test_tables_match_oracle(lib, n):
    out = [np.zeros(n), np.zeros(n), np.zeros((n, n)), np.zeros((n, n)), np.zeros((n, n)),
           np.zeros(n), np.zeros(n)]
    assert lib.kph_make_tables(n, *[P(a) for a in out]) == 0
    T = tables(n)
    for a, key in zip(out, ["x", "w", "D", "S", "K", "l0", "l1"]):
        assert np.max(np.abs(a - T[key])) <= 1e-12 * max(1.0, np.max(np.abs(T[key])))


@pytest.mark.parametrize("dim,n", [(2, 7), (3, 4)])
def test_blocks_match_oracle(lib, dim, n):
    params, _ = synth.mesh_params(3, dim, 9)
    N = n ** dim
    for rec in params[:4]:
        out = np.zeros((N, N))
        lib.kph_block(dim, n, P(rec), P(out))
        ref = element_block(rec, n, dim)
        assert np.max(np.abs(out - ref)) <= 1e-14 * np.max(np.abs(ref))


def host_setup(lib, dim, n, rec, block, rank=2):
    nf = 2 * rank if dim == 2 else 5
    f = np.zeros((nf, n, n))
    sig = np.zeros(4)
    steps = ctypes.c_int(0)
    st = lib.kph_setup(dim, n, rank, P(rec), P(block) if block is not None else None, None, P(f), P(sig),
                       ctypes.byref(steps))
    return st, f, sig


@pytest.mark.parametrize("dim,n,explicit", [(2, 6, True), (2, 6, False), (2, 12, True),
                                            (3, 4, True), (3, 4, False), (3, 6, False)])
def test_lanczos_setup_matches_full_svd(lib, dim, n, explicit):
    params, _ = synth.mesh_params(2, dim, 21)
    for rec in params[:3]:
        A = element_block(rec, n, dim)
        st, f, sig = host_setup(lib, dim, n, rec, A if explicit else None)
        assert st == 0
        fo = ksvd2d(A, n, 2) if dim == 2 else ksvd3d(A, n)
        so = fo["sigma"][:2] if dim == 2 else np.r_[fo["sigma1"][0], fo["sigma2"][:2]]
        got = sig[:2] if dim == 2 else sig[:3]
        assert np.max(np.abs(got / so - 1)) <= 1e-12
        assert rel(precond_matrix(factors_from_array(f, dim)), precond_matrix(fo)) <= 1e-12


@pytest.mark.parametrize("rank,n,explicit", [(1, 6, True), (1, 8, False), (3, 6, True),
                                             (3, 8, False), (3, 16, False)])
def test_lanczos_setup_rank1_rank3_2d(lib, rank, n, explicit):
    params = synth.draw_params(3, 2, 1002)
    for rec in params:
        A = element_block(rec, n, 2)
        st, f, sig = host_setup(lib, 2, n, rec, A if explicit else None, rank)
        assert st == 0
        fo = ksvd2d(A, n, rank)
        assert np.max(np.abs(sig[:rank] / fo["sigma"][:rank] - 1)) <= 1e-12
        assert rel(precond_matrix(factors_from_array(f, 2)), precond_matrix(fo)) <= 1e-12


@pytest.mark.parametrize("n", [2, 3, 6, 16, 31])
def test_real_schur(lib, n):
    rng = np.random.default_rng(n)
    for _ in range(5):
        C = rng.standard_normal((n, n))
        T = np.zeros((n, n))
        Q = np.zeros((n, n))
        assert lib.kph_schur(n, P(C), P(T), P(Q)) == 0
        assert rel(Q @ T @ Q.T, C) <= 1e-13
        assert np.max(np.abs(Q.T @ Q - np.eye(n))) <= 1e-13 * n
        assert np.all(np.tril(T, -2) == 0)
        for j in range(1, n):
            if T[j, j - 1] != 0:  # standardised 2x2 block: complex pair
                assert T[j, j] == T[j - 1, j - 1] and T[j - 1, j] * T[j, j - 1] < 0
                assert j < 2 or T[j - 1, j - 2] == 0
        ev = np.sort_complex(np.linalg.eigvals(C))
        assert np.max(np.abs(np.sort_complex(np.linalg.eigvals(T)) - ev)) <= 1e-10 * np.max(np.abs(ev))


@pytest.mark.parametrize("dim,n", [(2, 2), (2, 5), (2, 8), (2, 16), (2, 31), (3, 8)])
def test_apply_all_precisions(lib, dim, n):
    params, _ = synth.mesh_params(2, dim, 33)
    rng = np.random.default_rng(1)
    Z = {p: [] for p in range(4)}
    ZR = []
    for rec in params[:6]:
        fo = ksvd2d(element_block(rec, n, dim), n, 2) if dim == 2 else ksvd3d(element_block(rec, n, dim), n)
        F = factor_array(fo)
        tab = np.zeros((7 + n) * n * n)
        kinds = np.zeros(n, np.int8)
        assert lib.kph_form_tables(dim, n, 2, P(F), P(tab), P(kinds)) == 0
        r = rng.standard_normal(n ** dim)
        ZR.append(dense_solve(fo, r))
        for prec in range(4):
            z = np.zeros(n ** dim)
            lib.kph_apply(dim, n, prec, P(tab), P(kinds), P(r), P(z))
            Z[prec].append(z)
    for prec, tol in ((0, 1e-12), (1, 1e-5), (2, 2e-2), (3, 1e-4)):
        assert rel(np.array(Z[prec]), np.array(ZR)) <= tol, prec


@pytest.mark.parametrize("n,m", [(6, 8), (16, 8), (16, 3)])
def test_rank3_apply_all_precisions(lib, n, m):
    """2D rank 3: inner flexible GMRES on the three-term sum, preconditioned by
    the rank-2 apply, against the dense solve of the three-term P."""
    params = synth.draw_params(6, 2, 1002)
    rng = np.random.default_rng(5)
    Z = {p: [] for p in range(4)}
    ZR = []
    for rec in params:
        fo = ksvd2d(element_block(rec, n, 2), n, 3)
        F = factor_array(fo)
        assert F.shape[0] == 6
        tab = np.zeros((7 + n) * n * n)
        kinds = np.zeros(n, np.int8)
        assert lib.kph_form_tables(2, n, 2, P(np.ascontiguousarray(F[:4])), P(tab), P(kinds)) == 0
        r = rng.standard_normal(n * n)
        ZR.append(dense_solve(fo, r))
        for prec in range(4):
            z = np.zeros(n * n)
            it = lib.kph_apply_rank3(n, prec, P(F), P(tab), P(kinds), P(r), P(z), m)
            assert it > 0, (prec, it)
            Z[prec].append(z)
    for prec, tol in ((0, 1e-12), (1, 1e-5), (2, 2e-2), (3, 1e-4)):
        assert rel(np.array(Z[prec]), np.array(ZR)) <= tol, prec


def test_rank3_zero_rhs_and_exact_rank2(lib):
    """r = 0 gives z = 0 with no iterations; when A3 (x) B3 vanishes the first
    preconditioned step already solves the system (FP64)."""
    n = 6
    fo = ksvd2d(element_block(synth.draw_params(1, 2, 7)[0], n, 2), n, 3)
    F = factor_array(fo)
    tab = np.zeros((7 + n) * n * n)
    kinds = np.zeros(n, np.int8)
    assert lib.kph_form_tables(2, n, 2, P(np.ascontiguousarray(F[:4])), P(tab), P(kinds)) == 0
    z = np.ones(n * n)
    assert lib.kph_apply_rank3(n, 0, P(F), P(tab), P(kinds), P(np.zeros(n * n)), P(z), 8) == 0
    assert not z.any()
    F0 = F.copy()
    F0[4:] = 0.0
    fo0 = factors_from_array(F0, 2)
    r = np.random.default_rng(2).standard_normal(n * n)
    it = lib.kph_apply_rank3(n, 0, P(F0), P(tab), P(kinds), P(r), P(z), 8)
    assert 0 < it <= 2
    assert rel(z, dense_solve(fo0, r)) <= 1e-12


@pytest.mark.parametrize("n,explicit", [(8, True), (16, False), (16, True)])
def test_rank3_setup_then_apply_end_to_end(lib, n, explicit):
    """Rank-3 Lanczos setup (two-sided refinement of the third triplet), rank-2
    tables and the inner solve against the dense solve of the oracle's rank-3
    P: global <= 1e-12 (FP64), <= 1e-5 (FP32)."""
    params = synth.draw_params(12, 2, 1002)
    rng = np.random.default_rng(11)
    Z = {0: [], 1: []}
    ZR = []
    for rec in params:
        A = element_block(rec, n, 2)
        st, f, sig = host_setup(lib, 2, n, rec, A if explicit else None, 3)
        assert st == 0
        fo = ksvd2d(A, n, 3)
        assert np.max(np.abs(sig[:3] / fo["sigma"][:3] - 1)) <= 1e-12
        tab = np.zeros((7 + n) * n * n)
        kinds = np.zeros(n, np.int8)
        assert lib.kph_form_tables(2, n, 2, P(np.ascontiguousarray(f[:4])), P(tab), P(kinds)) == 0
        r = rng.standard_normal(n * n)
        ZR.append(dense_solve(fo, r))
        for prec in (0, 1):
            z = np.zeros(n * n)
            assert lib.kph_apply_rank3(n, prec, P(f), P(tab), P(kinds), P(r), P(z), 8) > 0
            Z[prec].append(z)
    assert rel(np.array(Z[0]), np.array(ZR)) <= 1e-12
    assert rel(np.array(Z[1]), np.array(ZR)) <= 1e-5


@pytest.mark.parametrize("dim,n,face", [(2, 6, False), (2, 8, True), (3, 4, True), (3, 5, False)])
def test_learned_judge_matches_oracle_accept(lib, dim, n, face):
    """The learned setup's judge (closed-form residuals of the prediction and
    of the SVD, the guard's power estimate through the SVD's apply tables)
    against oracle.mlp.accept on the same factors: the SVD's own factors,
    perturbations of several sizes, an all-zero prediction and a first factor
    made nearly singular."""
    from oracle import mlp as omlp
    params = synth.draw_params(3, dim, 41, face=face)
    rng = np.random.default_rng(7)
    lib.kph_learned_judge.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
    seen = set()
    for rec in params:
        A = element_block(rec, n, dim)
        fo = ksvd2d(A, n, 2) if dim == 2 else ksvd3d(A, n)
        F = np.ascontiguousarray(factor_array(fo))
        U, sv, Vt = np.linalg.svd(F[0])
        Fn = F.copy()
        Fn[0] = F[0] - (1.0 - 1e-6) * sv[-1] * np.outer(U[:, -1], Vt[-1])
        preds = [F, np.zeros_like(F), Fn]
        for pert in (1e-6, 0.01, 0.3):
            preds.append(F * (1.0 + pert * rng.standard_normal(F.shape)))
        for Fp in preds:
            Fp = np.ascontiguousarray(Fp)
            out = np.zeros(4)
            ok = lib.kph_learned_judge(dim, n, P(rec), P(Fp), P(F), 1.1, 0.1, P(out))
            ok_ref, rp, rs, g = omlp.accept(A, Fp, F, dim, guard=0.1)
            a = np.linalg.norm(A)
            assert out[2] == pytest.approx(a, rel=1e-13)
            assert abs(out[0] - rp) <= 1e-7 * a and abs(out[1] - rs) <= 1e-7 * a, (out, rp, rs)
            assert abs(out[3] - g) <= 1e-9 * max(1.0, g), (out[3], g)
            margin = min(abs(rp - 1.1 * rs) / a, abs(g - 0.1), abs(rp - a) / a)
            if margin > 1e-9:
                assert ok == int(ok_ref)
            seen.add(bool(ok))
    assert seen == {True, False}


@pytest.mark.parametrize("dim,n,mu", [(2, 5, 7), (2, 8, 10), (3, 4, 6), (3, 5, 5), (3, 6, 8)])
def test_quad_setup_matches_oracle(lib, dim, n, mu):
    """Setup of general (non-collocated quadrature) elements in the Gram form
    of the rearranged operator, host build, against the oracle's full SVD of
    the dense block assembled by its quadrature definition: sigma and P within
    1e-12."""
    from oracle import shuffled
    from oracle.ksvd import factors_from_array
    q = synth.quad_elements(3, dim, mu, seed=77)
    Q = shuffled.quad_tables(n, mu)
    lib.kph_setup_quad.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] + [ctypes.c_void_p] * 6
    for e in range(3):
        el = synth.quad_element(q, e, n)
        A = shuffled.element_block(el, Q)
        f = ksvd2d(A, n, 2) if dim == 2 else ksvd3d(A, n)
        so = f["sigma"][:2] if dim == 2 else np.r_[f["sigma1"][0], f["sigma2"][:2]]
        F = np.zeros((4 if dim == 2 else 5, n, n))
        sig = np.zeros(4)
        arrs = [np.ascontiguousarray(q[k][e]) for k in ("c", "a", "nu", "g")]
        st = lib.kph_setup_quad(dim, n, mu, q["tau"], *(P(x) for x in arrs), P(F), P(sig))
        assert st == 0
        assert np.max(np.abs(sig[:len(so)] / so - 1)) <= 1e-12
        Pg = precond_matrix(factors_from_array(F, dim))
        Po = precond_matrix(f)
        assert np.linalg.norm(Pg - Po) <= 1e-12 * np.linalg.norm(Po)


@pytest.mark.parametrize("nc,n", [(1, 5), (2, 4), (4, 4), (4, 8), (5, 6), (3, 8), (2, 16)])
def test_systems_setup_and_apply_match_oracle(lib, nc, n):
    """nc-component system blocks, host build: factors (sign included) and
    sigma against the oracle's full SVD of R(A) with nc n x nc n first factors,
    and P^{-1} r in FP64 and FP32 against the oracle's dense solve of P."""
    from oracle import systems
    m = nc * n
    sd = synth.systems_elements(2, nc, seed=11)
    lib.kph_sys_setup.argtypes = [ctypes.c_int] * 2 + [ctypes.c_void_p] * 5
    lib.kph_sys_apply.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p] * 4
    ne = 3 * m * m + 3 * n * n + n * m * m
    for e in range(2):
        A = np.ascontiguousarray(systems.element_block(sd, e, n))
        f = systems.ksvd_system(A, nc, n, 2)
        F = np.zeros(2 * m * m + 2 * n * n)
        sig = np.zeros(4)
        tab = np.zeros(ne)
        kinds = np.zeros(n, np.int8)
        assert lib.kph_sys_setup(nc, n, P(A), P(F), P(sig), P(tab), P(kinds)) == 0
        assert np.max(np.abs(sig[:2] / f["sigma"][:2] - 1)) <= 1e-12
        off = 0
        for j in range(2):
            Aj = F[off:off + m * m].reshape(m, m)
            Bj = F[off + m * m:off + m * m + n * n].reshape(n, n)
            off += m * m + n * n
            assert rel(Aj, f["A"][j]) <= 1e-10
            assert rel(Bj, f["B"][j]) <= 1e-10
        r = np.random.default_rng(e).standard_normal(m * n)
        zr = dense_solve(f, r)
        for prec, tol in ((0, 1e-12), (1, 5e-5)):
            z = np.zeros(m * n)
            lib.kph_sys_apply(nc, n, prec, P(tab), P(kinds), P(r), P(z))
            assert rel(z, zr) <= tol, (prec, rel(z, zr))
