"""KSVD tensor-product block-Jacobi preconditioner for very high order DG on MI355X.

The numerical work lives in libkp.so (HIP kernels for gfx950, C ABI in
include/kp.h); ``paper_1704_04549_amd.kp`` is its Python binding.
"""
__all__ = ["kp"]
