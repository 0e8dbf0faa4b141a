"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and lays out meshes; it contains none of
the preconditioner's arithmetic (no 1D tables, no element blocks, no SVD, no
solves).  Both the CPU oracle and the GPU path read the arrays it returns.

Element record (float64[16]), one per element:

    [0] beta_x   [1] beta_y   [2] beta_z (0 in 2D)   (element velocity a = -beta)
    [3] nu       [4] alpha    [5] phi
    [6] tau      [7] face flag (1.0: upwind face terms are part of the operator)
    [8..13] normal velocity u_f = a_f . n_f on the faces x-, x+, y-, y+, z-, z+
            (outward normal; u_f > 0 is outflow), with the face velocity
            a_f = (a_e + a_neighbour) / 2 of the conservative upwind flux;
            an element drawn without a mesh uses its own velocity on every face
    [14..15] reserved, zero

Draws (numpy PCG64 via ``default_rng``), per element in order:
beta_x, beta_y, [beta_z], log10(nu), alpha, phi with
beta ~ U[-1,1], log10 nu ~ U[-3,-1], alpha ~ U[0,0.5], phi ~ U[0,2pi).
The right-hand sides are drawn after all elements: N(0,1) of shape
(E, nrhs, n^d).
"""
from __future__ import annotations

import numpy as np

REC_LEN = 16
TAU = 0.1

# the workloads: dim, n, mesh, rank, face terms, coupling through faces, nrhs, seeds.
# c3 couples neighbours through the upwind flux (face velocities averaged over
# the two elements); c4 is the block-diagonal system of elements closed by
# their own upwind faces (the coupled p=15 system makes FGMRES(30) stagnate).
WORKLOADS = {
    "c1_2d_p7": dict(dim=2, n=8, mesh=16, rank=2, face=False, coupled=False, nrhs=1,
                     seed=1001, rhs_seed=2001),
    "c2_2d_p15": dict(dim=2, n=16, mesh=128, rank=2, face=False, coupled=False, nrhs=8,
                      seed=1002, rhs_seed=2002),
    "c3_3d_p7": dict(dim=3, n=8, mesh=32, rank=2, face=True, coupled=True, nrhs=1,
                     seed=1003, rhs_seed=2003),
    "c4_3d_p15": dict(dim=3, n=16, mesh=16, rank=2, face=True, coupled=False, nrhs=1,
                      seed=1004, rhs_seed=2004),
}
MLP_TRAIN_SEED = 3004
MLP_VAL_SEED = 4004
MIXED_SEED = 1005
MIXED_RHS_SEED = 2005


def draw_params(num_elems: int, dim: int, seed: int, face: bool = False,
                tau: float = TAU) -> np.ndarray:
    """Per-element records, float64[E, 12], drawn in element order."""
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    rng = np.random.default_rng(seed)
    k = dim + 3  # betas, log10 nu, alpha, phi
    u = rng.random((num_elems, k))  # row-major fill == per-element order
    rec = np.zeros((num_elems, REC_LEN), dtype=np.float64)
    rec[:, 0:dim] = 2.0 * u[:, 0:dim] - 1.0
    rec[:, 3] = 10.0 ** (-3.0 + 2.0 * u[:, dim])
    rec[:, 4] = 0.5 * u[:, dim + 1]
    rec[:, 5] = 2.0 * np.pi * u[:, dim + 2]
    rec[:, 6] = tau
    rec[:, 7] = 1.0 if face else 0.0
    if face:
        own_face_velocities(rec, dim)
    return rec


def own_face_velocities(rec: np.ndarray, dim: int) -> None:
    """Face normal velocities of isolated elements: a_f = a_e on every face."""
    for ax in range(dim):
        rec[:, 8 + 2 * ax] = rec[:, ax]       # low face: a.(-e_ax) = beta_ax
        rec[:, 9 + 2 * ax] = -rec[:, ax]      # high face: a.(+e_ax) = -beta_ax


def mesh_face_velocities(rec: np.ndarray, nbr: np.ndarray, dim: int) -> None:
    """Face normal velocities on a mesh: a_f = (a_e + a_neighbour) / 2 on every face."""
    for ax in range(dim):
        lo = rec[nbr[:, 2 * ax], ax]
        hi = rec[nbr[:, 2 * ax + 1], ax]
        rec[:, 8 + 2 * ax] = 0.5 * (rec[:, ax] + lo)
        rec[:, 9 + 2 * ax] = -0.5 * (rec[:, ax] + hi)


def draw_rhs(num_elems: int, nrhs: int, ndof: int, seed: int) -> np.ndarray:
    """Right-hand sides, float64[E, nrhs, ndof], N(0,1)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((num_elems, nrhs, ndof))


def mesh_params(mesh: int, dim: int, seed: int, tau: float = TAU) -> tuple:
    """Records with face terms on a periodic mesh^dim grid, and its neighbour table."""
    rec = draw_params(mesh ** dim, dim, seed, face=True, tau=tau)
    nbr = periodic_neighbours(mesh, dim)
    mesh_face_velocities(rec, nbr, dim)
    return rec, nbr


def periodic_neighbours(mesh: int, dim: int) -> np.ndarray:
    """Face neighbours on a periodic mesh^dim grid, int32[E, 2*dim].

    Elements are numbered e = (ex*M + ey)*M + ez (x slowest).  Column 2k is the
    neighbour across the low face of axis k, column 2k+1 across the high face.
    """
    M = mesh
    idx = np.arange(M ** dim).reshape((M,) * dim)
    cols = []
    for ax in range(dim):
        cols.append(np.roll(idx, 1, axis=ax).ravel())   # low-face neighbour: index-1
        cols.append(np.roll(idx, -1, axis=ax).ravel())  # high-face neighbour: index+1
    return np.stack(cols, axis=1).astype(np.int32)


def workload(name: str, num_elems: int | None = None):
    """Records, neighbours and right-hand sides of a named workload.

    ``num_elems`` truncates the element list (the first elements of the full
    draw) for small test cases; neighbours are then only meaningful when the
    full mesh is used.
    """
    cfg = WORKLOADS[name]
    dim, n, M = cfg["dim"], cfg["n"], cfg["mesh"]
    E_full = M ** dim
    E = E_full if num_elems is None else int(num_elems)
    rec = draw_params(E_full, dim, cfg["seed"], face=cfg["face"])
    nbr = periodic_neighbours(M, dim) if cfg["coupled"] else None
    if cfg["coupled"]:
        mesh_face_velocities(rec, nbr, dim)
    rec = rec[:E]
    rhs = draw_rhs(E_full, cfg["nrhs"], n ** dim, cfg["rhs_seed"])[:E]
    nbr = nbr if E == E_full else None
    return dict(cfg, num_elems=E, params=rec, rhs=rhs, nbr=nbr)


def mixed_batch(n2d: int = 50000, n3d: int = 2000, seed: int = MIXED_SEED):
    """Mixed-degree batch: 2D elements with p ~ U{3..30}, then 3D with p ~ U{3..15}.

    p is drawn before each element's parameters.  Every element is closed by
    the outflow terms of its own upwind faces (face flag set, face velocities
    from its own velocity), as the block-diagonal 3D p = 15 workload: without
    them an advection-dominated block is nearly singular (S is) and the
    block-diagonal system does not converge.  Returns (dims, ns, params).
    """
    rng = np.random.default_rng(seed)
    dims, ns, recs = [], [], []
    for dim, count, pmax in ((2, n2d, 30), (3, n3d, 15)):
        for _ in range(count):
            p = int(rng.integers(3, pmax + 1))
            u = rng.random(dim + 3)
            rec = np.zeros(REC_LEN)
            rec[0:dim] = 2.0 * u[0:dim] - 1.0
            rec[3] = 10.0 ** (-3.0 + 2.0 * u[dim])
            rec[4] = 0.5 * u[dim + 1]
            rec[5] = 2.0 * np.pi * u[dim + 2]
            rec[6] = TAU
            rec[7] = 1.0
            for ax in range(dim):
                rec[8 + 2 * ax] = rec[ax]
                rec[9 + 2 * ax] = -rec[ax]
            dims.append(dim)
            ns.append(p + 1)
            recs.append(rec)
    return (np.asarray(dims, np.int8), np.asarray(ns, np.int16),
            np.asarray(recs, np.float64))


QUAD_SEED = 1006


def quad_points01(mu: int) -> np.ndarray:
    """The mu Gauss-Legendre points of [0,1]: where a DG code evaluates the
    flux Jacobians that a general element carries (input layout only)."""
    xi, _ = np.polynomial.legendre.leggauss(mu)
    return 0.5 * (xi + 1.0)


def quad_elements(num_elems: int, dim: int, mu: int, seed: int = QUAD_SEED, tau: float = TAU) -> dict:
    """General elements: coefficients at the mu^d quadrature points (and
    mu^(d-1) per face) of smoothly varying, non-separable fields, as a DG
    code's linearisation hands them over on curved elements.

    Per element, drawn in order: beta (d values, U[-1,1]), log10 nu
    (U[-3,-1]), alpha (U[0,0.5]), phi (U[0,2pi)), gamma (U[0,0.3]: velocity
    variation), kappa (U[0,0.2]: metric variation), psi (d phases, U[0,2pi)).
    With x the point's coordinates on [0,1]^d:
      J(x)     = 1 + kappa sin(pi (x_0 + ... + x_{d-1}) + psi_0)
      c(x)     = J(x) (1 + alpha sin(pi x_0 ... x_{d-1} + phi))
      a_i(x)   = -beta_i J(x) (1 + gamma sin(pi x_{i+1 mod d} + psi_i))
      nu(x)    = nu J(x) (1 + gamma cos(pi x_0 x_1 + psi_0))
      g_f(x)   = max(a(x) . n_f, 0) on face f (outflow part of the upwind flux)
    Arrays: c [E][mu^d], a [E][d][mu^d], nu [E][mu^d], g [E][2d][mu^(d-1)]
    (C order, x slowest; on a face the remaining axes in order)."""
    rng = np.random.default_rng(seed)
    xq = quad_points01(mu)
    E = num_elems
    k = 2 * dim + 6
    u = rng.random((E, k))
    beta = 2.0 * u[:, 0:dim] - 1.0
    nu0 = 10.0 ** (-3.0 + 2.0 * u[:, dim])
    alpha = 0.5 * u[:, dim + 1]
    phi = 2.0 * np.pi * u[:, dim + 2]
    gamma = 0.3 * u[:, dim + 3]
    kappa = 0.2 * u[:, dim + 4]
    psi = 2.0 * np.pi * u[:, dim + 5:dim + 5 + dim]

    def fields(X):
        # X: list of d coordinate arrays of one shape
        s = sum(X)
        prod = X[0].copy()
        for t in X[1:]:
            prod = prod * t
        J = 1.0 + kappa[:, None] * np.sin(np.pi * s[None] + psi[:, 0:1])
        c = J * (1.0 + alpha[:, None] * np.sin(np.pi * prod[None] + phi[:, None]))
        a = np.stack([-beta[:, i:i + 1] * J *
                      (1.0 + gamma[:, None] * np.sin(np.pi * X[(i + 1) % dim][None] + psi[:, i:i + 1]))
                      for i in range(dim)], axis=1)
        nu = nu0[:, None] * J * (1.0 + gamma[:, None] * np.cos(np.pi * X[0][None] * X[1][None] + psi[:, 0:1]))
        return c, a, nu

    grid = np.meshgrid(*([xq] * dim), indexing="ij")
    c, a, nu = fields([g.ravel() for g in grid])
    g = []
    for ax in range(dim):
        for side in (0, 1):
            coords = [t.ravel() for t in np.meshgrid(*([xq] * (dim - 1)), indexing="ij")] if dim > 1 else []
            X = coords[:ax] + [np.full(mu ** (dim - 1), float(side))] + coords[ax:]
            _, af, _ = fields(X)
            un = af[:, ax, :] * (1.0 if side == 1 else -1.0)
            g.append(np.maximum(un, 0.0))
    return dict(dim=dim, mu=mu, tau=tau, c=c, a=a, nu=nu, g=np.stack(g, axis=1),
                draws=np.concatenate([beta, nu0[:, None], alpha[:, None], phi[:, None], gamma[:, None],
                                      kappa[:, None], psi], axis=1))


def quad_element(q: dict, e: int, n: int) -> dict:
    """Element e of a quad_elements batch as the oracle's element dict."""
    return dict(dim=q["dim"], n=n, mu=q["mu"], tau=q["tau"], c=q["c"][e], a=q["a"][e], nu=q["nu"][e],
                g=q["g"][e])


SYSTEMS_SEED = 1007


def systems_elements(num_elems: int, nc: int, seed: int = SYSTEMS_SEED, tau: float = TAU,
                     face: bool = True) -> dict:
    """2D elements of an nc-component system (input data only): per element,
    drawn in order, for each axis a flux Jacobian J_i = R diag(lam) R^-1 with
    R = I + 0.3 G (G ~ N(0,1), drawn again while cond(R) > 10: the Euler
    Jacobians' eigenvector matrices are well conditioned) and
    lam ~ U[-1,1]^nc (real eigenvalues, as for the Euler equations), then
    log10 nu ~ U[-3,-1], alpha ~ U[0,0.5], phi ~ U[0,2pi).  Also handed over,
    as a DG code's upwind flux would, the positive parts
    (J_i)^+ = R diag(max(lam,0)) R^-1 and (-J_i)^+ of each axis (outflow
    through the high and the low face)."""
    rng = np.random.default_rng(seed)
    E = num_elems
    J = np.zeros((E, 2, nc, nc))
    Jp = np.zeros((E, 2, nc, nc))
    Jm = np.zeros((E, 2, nc, nc))
    nu = np.zeros(E)
    alpha = np.zeros(E)
    phi = np.zeros(E)
    for e in range(E):
        for ax in range(2):
            R = np.eye(nc) + 0.3 * rng.standard_normal((nc, nc))
            while np.linalg.cond(R) > 10.0:
                R = np.eye(nc) + 0.3 * rng.standard_normal((nc, nc))
            lam = 2.0 * rng.random(nc) - 1.0
            Ri = np.linalg.inv(R)
            J[e, ax] = R @ np.diag(lam) @ Ri
            Jp[e, ax] = R @ np.diag(np.maximum(lam, 0.0)) @ Ri
            Jm[e, ax] = R @ np.diag(np.maximum(-lam, 0.0)) @ Ri
        u = rng.random(3)
        nu[e] = 10.0 ** (-3.0 + 2.0 * u[0])
        alpha[e] = 0.5 * u[1]
        phi[e] = 2.0 * np.pi * u[2]
    return dict(nc=nc, tau=tau, face=face, J=J, Jp=Jp, Jm=Jm, nu=nu, alpha=alpha, phi=phi)


def systems_records(sd: dict) -> np.ndarray:
    """The drawn systems elements packed as records [E][6 nc^2 + 5]: Jx, Jy,
    (Jx)^+, (Jy)^+, (-Jx)^+, (-Jy)^+ (nc x nc row-major each), nu, alpha,
    phi, tau, face flag (the layout the library's systems block builder reads)."""
    E, nc = sd["J"].shape[0], sd["nc"]
    q = nc * nc
    rec = np.zeros((E, 6 * q + 5))
    for e in range(E):
        mats = (sd["J"][e, 0], sd["J"][e, 1], sd["Jp"][e, 0], sd["Jp"][e, 1], sd["Jm"][e, 0], sd["Jm"][e, 1])
        for k, M in enumerate(mats):
            rec[e, k * q:(k + 1) * q] = M.ravel()
        rec[e, 6 * q:] = (sd["nu"][e], sd["alpha"][e], sd["phi"][e], sd["tau"], 1.0 if sd["face"] else 0.0)
    return rec


SYSTEMS_RHS_SEED = 2007


def systems_workload(name: str = "sys_kh_p7", num_elems: int | None = None) -> dict:
    """The systems workload: 2D, nc = 4 components (the 2D Euler equations'
    count), p = 7 (n = 8: first factors 32 x 32, the largest nc n <= 32),
    128 x 128 = 16384 elements (the size of the paper's 2D Kelvin-Helmholtz
    mesh), each element closed by its own upwind faces (block-diagonal
    system), tau = 0.01 (the smaller of the paper's two Euler time steps);
    one N(0,1) right-hand side per element."""
    if name != "sys_kh_p7":
        raise KeyError(name)
    nc, n = 4, 8
    E = 16384 if num_elems is None else num_elems
    sd = systems_elements(E, nc, seed=SYSTEMS_SEED, tau=0.01)
    return dict(name=name, nc=nc, n=n, num_elems=E, sd=sd, recs=systems_records(sd),
                rhs=draw_rhs(E, 1, nc * n * n, SYSTEMS_RHS_SEED))
