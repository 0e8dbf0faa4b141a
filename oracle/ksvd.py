"""Kronecker-product SVD by its plain definition (Sec. 4.1, eq. NKP).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Van Loan rearrangement: for A of size (m1*m2) x (n1*n2) viewed as an
m1 x n1 grid of m2 x n2 blocks A_ij, the rearranged matrix has one row per
block, holding that block flattened, so that
  || A - sum_j A_j (x) B_j ||_F = || R(A) - sum_j vec(A_j) vec(B_j)^T ||_F.
Here vec flattens row-major (the paper stacks columns; any fixed bijection
gives the same singular values and, after un-flattening, the same factors).
With that convention the row of block (i, j) is i*n1 + j and the column of
entry (k, l) is k*n2 + l.

The best rank-r approximation is read off a full LAPACK SVD:
vec(A_j) = sqrt(sigma_j) u_j, vec(B_j) = sqrt(sigma_j) v_j (Sec. 4.1, KSVD).

3D uses the two-stage form of Sec. 4.3.1: A ~ A1 (x) D1 (rank 1 of the
n^2 x n^4 rearrangement), then D1 ~ B1 (x) C1 + B2 (x) C2 (rank 2 of R(D1)),
giving P = A1 (x) B1 (x) C1 + A1 (x) B2 (x) C2 (eq. 3d-simple-precond).

Split axis (Sec. 4.3.1 splits the first factor; which axis carries the rank-1
stage is a choice the paper does not vary): ``ksvd3d_axis`` runs the two-stage
KSVD on the block with its tensor axes relabelled so that the chosen axis comes
first (orders x,y,z; y,x,z; z,x,y), and ``precond_matrix`` maps P back;
``ksvd3d_best_axis`` takes the axis whose rank-1 stage keeps the most of
||A||_F (the largest stage-1 sigma_1; ties to the lowest axis).

Canonical sign: the pair (u_j, v_j) -> (-u_j, -v_j) leaves P unchanged, so
each u_j is flipped to make its largest-magnitude entry (lowest index on
ties) positive.

Pinned by tests/test_oracle_ksvd.py (index formula by loops, rank-1 recovery,
Eckart-Young residual, exact separable cases, the relabelling by loops, a block
separable only along y or z recovered exactly by its own axis and not by the
first).
"""
from __future__ import annotations

import numpy as np


def rearrange(A: np.ndarray, m1: int, n1: int, m2: int, n2: int) -> np.ndarray:
    """R(A): (m1*n1) x (m2*n2), row i*n1+j = block (i,j) flattened row-major."""
    assert A.shape == (m1 * m2, n1 * n2)
    return A.reshape(m1, m2, n1, n2).transpose(0, 2, 1, 3).reshape(m1 * n1, m2 * n2)


def canonical_sign(u: np.ndarray) -> float:
    k = int(np.argmax(np.abs(u)))
    return 1.0 if u[k] >= 0.0 else -1.0


def ksvd(A: np.ndarray, m1: int, n1: int, m2: int, n2: int, r: int):
    """Best r-term sum_j A_j (x) B_j by the full SVD of R(A).

    Returns (sigma_all, [A_j], [B_j]) with sigma_all every singular value.
    """
    R = rearrange(A, m1, n1, m2, n2)
    U, s, Vt = np.linalg.svd(R, full_matrices=False)
    As, Bs = [], []
    for j in range(r):
        sg = canonical_sign(U[:, j])
        u = sg * U[:, j]
        v = sg * Vt[j]
        As.append(np.sqrt(s[j]) * u.reshape(m1, n1))
        Bs.append(np.sqrt(s[j]) * v.reshape(m2, n2))
    return s, As, Bs


def ksvd2d(A: np.ndarray, n: int, r: int = 2) -> dict:
    s, As, Bs = ksvd(A, n, n, n, n, r)
    return dict(dim=2, n=n, rank=r, sigma=s, A=As, B=Bs)


def ksvd3d(A: np.ndarray, n: int) -> dict:
    """Two-stage 3D KSVD (Alg. 7, first two steps)."""
    s1, A1, D1 = ksvd(A, n, n, n * n, n * n, 1)
    s2, Bs, Cs = ksvd(D1[0], n, n, n, n, 2)
    return dict(dim=3, n=n, rank=2, sigma1=s1, sigma2=s2,
                A1=A1[0], D1=D1[0], B=Bs, C=Cs)


# axis orders of the 3D split: the chosen axis first, the other two in order
AXIS_ORDERS = {0: (0, 1, 2), 1: (1, 0, 2), 2: (2, 0, 1)}


def permute_block(A: np.ndarray, n: int, order) -> np.ndarray:
    """The 3D block with its tensor axes relabelled: axis q of the result is
    axis order[q] of A (rows and columns alike; C order, first axis slowest)."""
    A6 = A.reshape((n,) * 6)
    return A6.transpose(*order, *(3 + q for q in order)).reshape(n ** 3, n ** 3)


def inverse_order(order):
    inv = [0, 0, 0]
    for q, o in enumerate(order):
        inv[o] = q
    return tuple(inv)


def ksvd3d_axis(A: np.ndarray, n: int, axis: int) -> dict:
    """Two-stage KSVD with the rank-1 stage on `axis` (factors in the
    relabelled frame; precond_matrix maps P back)."""
    f = ksvd3d(permute_block(A, n, AXIS_ORDERS[axis]), n)
    f["axis"] = axis
    return f


def ksvd3d_best_axis(A: np.ndarray, n: int) -> dict:
    fs = [ksvd3d_axis(A, n, k) for k in range(3)]
    k = int(np.argmax([f["sigma1"][0] for f in fs]))
    return fs[k]


def ksvd3d_rearranged(R1: np.ndarray, n: int) -> dict:
    """ksvd3d from the stage-1 rearranged matrix R(A) (n^2 x n^4) itself, for
    blocks too large to form densely: the same full SVDs."""
    U, s1, Vt = np.linalg.svd(R1, full_matrices=False)
    sg = canonical_sign(U[:, 0])
    A1 = np.sqrt(s1[0]) * sg * U[:, 0].reshape(n, n)
    D1 = np.sqrt(s1[0]) * sg * Vt[0].reshape(n * n, n * n)
    s2, Bs, Cs = ksvd(D1, n, n, n, n, 2)
    return dict(dim=3, n=n, rank=2, sigma1=s1, sigma2=s2, A1=A1, D1=D1, B=Bs, C=Cs)


def precond_matrix(f: dict) -> np.ndarray:
    """Dense P assembled from the factors (eqs. 2d-kron-sum, 3d-simple-precond),
    in the block's own axis order."""
    if f["dim"] == 2:
        return sum(np.kron(a, b) for a, b in zip(f["A"], f["B"]))
    A1 = f["A1"]
    P = sum(np.kron(A1, np.kron(b, c)) for b, c in zip(f["B"], f["C"]))
    axis = f.get("axis", 0)
    if axis:
        P = permute_block(P, f["n"], inverse_order(AXIS_ORDERS[axis]))
    return P


def factor_array(f: dict) -> np.ndarray:
    """Factors packed as a float64[k, n, n] stack.

    2D rank r: [A_1, B_1, A_2, B_2, ...]; 3D: [A1, B1, C1, B2, C2].
    """
    if f["dim"] == 2:
        mats = []
        for a, b in zip(f["A"], f["B"]):
            mats += [a, b]
        return np.stack(mats)
    return np.stack([f["A1"], f["B"][0], f["C"][0], f["B"][1], f["C"][1]])


def factors_from_array(arr: np.ndarray, dim: int) -> dict:
    n = arr.shape[-1]
    if dim == 2:
        r = arr.shape[0] // 2
        return dict(dim=2, n=n, rank=r, A=[arr[2 * j] for j in range(r)],
                    B=[arr[2 * j + 1] for j in range(r)])
    return dict(dim=3, n=n, rank=2, A1=arr[0], B=[arr[1], arr[3]], C=[arr[2], arr[4]])
