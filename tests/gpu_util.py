"""Helpers shared by the GPU tests: device batches from the seeded workloads."""
import numpy as np
import torch

from paper_1704_04549_amd import kp

DEV = torch.device("cuda", 0)


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def batch(params, dim, n, blocks=None, nbr=None):
    return kp.Batch(to_dev(params), dim, n,
                    blocks=to_dev(blocks) if blocks is not None and not torch.is_tensor(blocks) else blocks,
                    nbr=to_dev(nbr) if nbr is not None else None)


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def align_sign(f_gpu, f_ref):
    """Factors of one term are defined up to a joint sign; align to the reference."""
    s = np.sign(np.sum(f_gpu * f_ref))
    return f_gpu * (s if s != 0 else 1.0)
