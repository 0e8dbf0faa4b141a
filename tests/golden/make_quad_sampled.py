"""Write quad_sampled.npz: the oracle's two-stage KSVD and preconditioner solves
of three general 3D elements with n = 16 basis nodes and mu = 17 quadrature
points per axis (non-collocated quadrature, Sec. 3.4.1), elements 0, 100 and
255 of synth.quad_elements(256, 3, 17) (seed 1006).

Calls only oracle/ and the seeded generator: R(A) (256 x 65536) row by row from
the shuffled transpose products (Sec. 4.3.2), full SVDs of it and of R(D1)
(Sec. 4.3.1), and z = P^{-1} r by dense LU of P for r drawn with seed 2006.
Stored: element indices, the singular values (stage 1 sigma_1, stage 2
sigma_1, sigma_2), z.  About a minute.

Usage: python tests/golden/make_quad_sampled.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import shuffled  # noqa: E402
from oracle.apply import dense_solve  # noqa: E402
from oracle.ksvd import ksvd3d_rearranged  # noqa: E402

N, MU, E, IDX, RHS_SEED = 16, 17, 256, (0, 100, 255), 2006


def main():
    q = synth.quad_elements(E, 3, MU)
    Q = shuffled.quad_tables(N, MU)
    r = np.random.default_rng(RHS_SEED).standard_normal((E, N ** 3))
    sig, z = [], []
    for e in IDX:
        el = synth.quad_element(q, e, N)
        f = ksvd3d_rearranged(shuffled.rearranged_rows(el, Q), N)
        sig.append(np.r_[f["sigma1"][0], f["sigma2"][:2]])
        z.append(dense_solve(f, r[e]))
    np.savez_compressed(os.path.join(HERE, "quad_sampled.npz"), idx=np.array(IDX), sigma=np.stack(sig),
                        z=np.stack(z), n=N, mu=MU, num_elems=E, rhs_seed=RHS_SEED)


if __name__ == "__main__":
    main()
