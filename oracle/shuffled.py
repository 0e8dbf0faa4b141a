"""General (non-collocated) element blocks and the sum-factorised shuffled
products of the rearranged block (Sec. 3.4.1, eq. jac-entries; Sec. 4.2.1 and
Sec. 4.3.2).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A general element carries its data at mu >= n Gauss-Legendre quadrature points
per axis of [0,1] (the points where a DG code evaluates its flux Jacobians):
  c[q]        mass coefficient (|det J| times the pointwise mass factor),
  a[i][q]     flux Jacobian component dF_i/du (i = 0..d-1),
  nu[q]       coefficient of the second-order term,
  g[f][q']    upwind face coefficient dF^/du^- on face f = 2*axis + side at
              the face's own quadrature points (mu^(d-1) of them),
with tau the time-step factor.  Basis: Lagrange on the n Gauss-Legendre nodes;
Phi[alpha, j] = phi_j(x_alpha), dPhi[alpha, j] = phi_j'(x_alpha) at the mu
quadrature points.  Rows of the block are test functions, columns trial
functions, C order with x slowest.  The block is (eq. jac-entries with F = a u,
the mass of eq. M-entries, and a nu grad.grad term):

  A = sum_q w_q c_q phi_I phi_K
      - tau sum_i sum_q w_q a_i(q) (d_i phi_I) phi_K
      + tau sum_i sum_q w_q nu_q (d_i phi_I) (d_i phi_K)
      + tau sum_f sum_{q' on f} w_q' g_f(q') phi_I phi_K.

Every piece is one "term": per axis a pair (L, R) of point-by-basis matrices
(test side, trial side) over that axis's points, and a coefficient tensor f
over the product of the axes' points, weights included, so that
  A_term = (L_x (x) L_y [(x) L_z])^T diag(vec f) (R_x (x) R_y [(x) R_z]).
A face term uses the single point l_s = phi(0) or phi(1) on its own axis.

``element_block`` assembles A by that plain definition (dense Kronecker
products).  ``shuffled_matvec`` / ``shuffled_rmatvec`` compute R(A) v and
R(A)^T u without forming A, by the sum factorisation of Sec. 4.2.1 (2D) and
Sec. 4.3.2 (3D stage 1, A ~ A1 (x) D1), each counting its operations in a
``Flops`` counter: O(p^3) per product in 2D and O(p^5) in 3D, where the
innermost contraction over the n^4 right vector has four free indices.

With mu = n the basis is collocated (Phi = I, dPhi = D) and constant
coefficients give the blocks of ``oracle.blocks``.

Pinned by tests/test_oracle_shuffled.py (collocated reduction to the
structured generator's block, exact integration of polynomial data for every
mu >= n, the shuffled products against the explicit rearrangement, and the
operation counts' growth in n).
"""
from __future__ import annotations

import numpy as np

from .apply import Flops
from .ksvd import rearrange
from .tables import gauss_legendre01, lagrange_values


def lagrange_derivative_values(x: np.ndarray, t: float) -> np.ndarray:
    """phi_j'(t) for the Lagrange basis on nodes x, at any point t (product rule)."""
    n = len(x)
    out = np.zeros(n)
    for j in range(n):
        den = 1.0
        for k in range(n):
            if k != j:
                den *= x[j] - x[k]
        s = 0.0
        for m in range(n):
            if m == j:
                continue
            p = 1.0
            for k in range(n):
                if k != j and k != m:
                    p *= t - x[k]
            s += p
        out[j] = s / den
    return out


def quad_tables(n: int, mu: int) -> dict:
    """Basis values and derivatives at the mu-point Gauss-Legendre rule of [0,1]."""
    xn, _ = gauss_legendre01(n)
    xq, wq = gauss_legendre01(mu)
    Phi = np.stack([lagrange_values(xn, t) for t in xq])
    dPhi = np.stack([lagrange_derivative_values(xn, t) for t in xq])
    return dict(n=n, mu=mu, xn=xn, xq=xq, wq=wq, Phi=Phi, dPhi=dPhi,
                l0=lagrange_values(xn, 0.0), l1=lagrange_values(xn, 1.0))


def _outer(*vs):
    out = vs[0]
    for v in vs[1:]:
        out = np.multiply.outer(out, v)
    return out


def terms(el: dict, Q: dict) -> list:
    """The block's terms: (list of (L, R) per axis, coefficient tensor f)."""
    dim, tau = el["dim"], el["tau"]
    mu = Q["mu"]
    P, dP, w = Q["Phi"], Q["dPhi"], Q["wq"]
    shape = (mu,) * dim
    wd = _outer(*([w] * dim))
    out = [([(P, P)] * dim, wd * el["c"].reshape(shape))]
    for i in range(dim):
        lr = [(P, P)] * dim
        lr[i] = (dP, P)
        out.append((lr, -tau * wd * el["a"][i].reshape(shape)))
    for i in range(dim):
        lr = [(P, P)] * dim
        lr[i] = (dP, dP)
        out.append((lr, tau * wd * el["nu"].reshape(shape)))
    wf = _outer(*([w] * (dim - 1))) if dim > 1 else np.ones(())
    for i in range(dim):
        for s, l in ((0, Q["l0"]), (1, Q["l1"])):
            lr = [(P, P)] * dim
            lr[i] = (l[None, :], l[None, :])
            f = tau * wf * el["g"][2 * i + s].reshape((mu,) * (dim - 1))
            out.append((lr, np.expand_dims(f, i)))
    return out


def _kron(ms):
    out = ms[0]
    for m in ms[1:]:
        out = np.kron(out, m)
    return out


def element_block(el: dict, Q: dict) -> np.ndarray:
    """Dense n^d x n^d block by the plain quadrature definition."""
    A = 0.0
    for lr, f in terms(el, Q):
        L = _kron([p[0] for p in lr])
        R = _kron([p[1] for p in lr])
        A = A + L.T @ (f.reshape(-1)[:, None] * R)
    return A


def _ein(spec, a, b, k, fc):
    """einsum of two operands contracting one index of length k: (2k - 1)
    operations per output entry (k when nothing is summed)."""
    out = np.einsum(spec, a, b)
    fc.add(out.size * max(2 * k - 1, 1))
    return out


def shuffled_matvec(el: dict, Q: dict, v: np.ndarray, fc: Flops | None = None) -> np.ndarray:
    """u = R(A) v: 2D R is n^2 x n^2 (rows (x test, x trial), columns (y test,
    y trial)); 3D stage 1 R is n^2 x n^4 (columns ((y,z) test, (y,z) trial))."""
    fc = fc if fc is not None else Flops()
    n, dim = el["n"], el["dim"]
    u = np.zeros((n, n))
    for lr, f in terms(el, Q):
        (Lx, Rx) = lr[0]
        if dim == 2:
            (Ly, Ry) = lr[1]
            V = v.reshape(n, n)                                  # [b, d]
            t = _ein("bd,qd->bq", V, Ry, n, fc)                  # sum_d R_y[q, d] v[b, d]
            s = _ein("qb,bq->q", Ly, t, n, fc)                   # s[beta]
            q = _ein("pq,q->p", f, s, f.shape[1], fc)            # q[alpha]
        else:
            (Ly, Ry), (Lz, Rz) = lr[1], lr[2]
            V = v.reshape(n, n, n, n)                            # [b, e, d, g]
            t1 = _ein("bedg,rg->bedr", V, Rz, n, fc)             # four free indices: O(n^4 mu)
            t2 = _ein("re,bedr->bdr", Lz, t1, n, fc)
            t3 = _ein("qd,bdr->bqr", Ry, t2, n, fc)
            s = _ein("qb,bqr->qr", Ly, t3, n, fc)                # s[beta, gamma]
            q = _ein("pqr,qr->p", f, s, s.size, fc)
        lq = Lx * q[:, None]
        fc.add(lq.size)
        u += _ein("pa,pc->ac", lq, Rx, Lx.shape[0], fc)
        fc.add(u.size)
    return u.reshape(-1)


def shuffled_rmatvec(el: dict, Q: dict, u: np.ndarray, fc: Flops | None = None) -> np.ndarray:
    """v = R(A)^T u (the transpose product, the same factorisation read backwards)."""
    fc = fc if fc is not None else Flops()
    n, dim = el["n"], el["dim"]
    U = u.reshape(n, n)
    v = np.zeros((n,) * (2 * (dim - 1)))
    for lr, f in terms(el, Q):
        (Lx, Rx) = lr[0]
        t = _ein("pa,ac->pc", Lx, U, n, fc)
        q = _ein("pc,pc->p", t, Rx, n, fc)                       # q[alpha]
        if dim == 2:
            (Ly, Ry) = lr[1]
            s = _ein("pq,p->q", f, q, f.shape[0], fc)            # s[beta]
            ls = Ly * s[:, None]
            fc.add(ls.size)
            v += _ein("qb,qd->bd", ls, Ry, Ly.shape[0], fc)
        else:
            (Ly, Ry), (Lz, Rz) = lr[1], lr[2]
            s = _ein("pqr,p->qr", f, q, f.shape[0], fc)          # s[beta, gamma]
            t3 = _ein("qb,qr->bqr", Ly, s, 1, fc)
            t2 = _ein("bqr,qd->bdr", t3, Ry, Ry.shape[0], fc)
            t1 = _ein("bdr,re->bedr", t2, Lz, 1, fc)
            v += _ein("bedr,rg->bedg", t1, Rz, Rz.shape[0], fc)  # four free indices
        fc.add(v.size)
    return v.reshape(-1)


def explicit_rearranged(el: dict, Q: dict) -> np.ndarray:
    """R(A) of the dense block (2D: n^2 x n^2; 3D stage 1: n^2 x n^4)."""
    n, dim = el["n"], el["dim"]
    A = element_block(el, Q)
    if dim == 2:
        return rearrange(A, n, n, n, n)
    return rearrange(A, n, n, n * n, n * n)


def rearranged_rows(el: dict, Q: dict) -> np.ndarray:
    """R(A) (3D stage 1: n^2 x n^4) row by row, each row R(A)^T e_i by the
    shuffled transpose product, without forming the block."""
    n = el["n"]
    m = n * n
    rows = []
    for i in range(m):
        e = np.zeros(m)
        e[i] = 1.0
        rows.append(shuffled_rmatvec(el, Q, e))
    return np.stack(rows)
