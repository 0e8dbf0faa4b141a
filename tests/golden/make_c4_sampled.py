"""Write c4_sampled.npz: the oracle's KSVD and preconditioner solves on 64
elements spread evenly over the 3D p = 15 workload (4096 elements, n = 16).

Calls only oracle/ and the seeded generator (synth): per element the block by
its definition, the two-stage KSVD by full SVDs (Sec. 4.3.1), and
z = P^{-1} r by the Schur route (Algs. 7-8), which the oracle's tests pin to
the dense solve.  Stored: element indices, the singular values (stage 1
sigma_1, stage 2 sigma_1, sigma_2) and z for the workload's first right-hand
side.  About a minute on 8 cores.

Usage: python tests/golden/make_c4_sampled.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

NUM = 64


def one(e):
    from threadpoolctl import threadpool_limits

    import synth
    from oracle.apply import SchurPrecond
    from oracle.blocks import element_block
    from oracle.ksvd import ksvd3d
    w = synth.workload("c4_3d_p15")
    with threadpool_limits(limits=1):
        A = element_block(w["params"][e], 16, 3)
        f = ksvd3d(A, 16)
        z = SchurPrecond(f).solve(w["rhs"][e, 0])
    return e, np.r_[f["sigma1"][0], f["sigma2"][:2]], z


def main():
    import multiprocessing as mp
    idx = np.linspace(0, 4095, NUM).round().astype(int)
    with mp.get_context("spawn").Pool(min(8, os.cpu_count() or 1)) as pool:
        res = sorted(pool.map(one, idx.tolist()))
    np.savez_compressed(os.path.join(HERE, "c4_sampled.npz"), idx=np.array([r[0] for r in res]),
                        sigma=np.stack([r[1] for r in res]), z=np.stack([r[2] for r in res]))


if __name__ == "__main__":
    main()
