"""Python binding of the libkp C ABI (include/kp.h): argument marshalling only.

Every entry point keeps its C name and order of arguments; device buffers are
passed as torch tensors on the context's device (their data pointers are
handed to the library).  All numerical work runs in the HIP kernels of
libkp.so; this module raises if the library is missing and has no CPU path.
A non-OK status raises ``KpError``.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkp.so")

KP_OK, KP_ERR_ARG, KP_ERR_ALLOC, KP_ERR_HIP, KP_ERR_NUMERIC, KP_ERR_NOCONV, KP_ERR_UNSUPPORTED = range(7)
KP_FP64, KP_FP32, KP_BF16, KP_BF16X3 = 0, 1, 2, 3
KP_SETUP_SVD, KP_SETUP_LEARNED, KP_SETUP_LEARNED_WARM = 0, 1, 2
KP_PC_NONE, KP_PC_KSVD, KP_PC_BJ = 0, 1, 2
KP_OPT_FGMRES_GRAPHS, KP_OPT_APPLY_MFMA16, KP_OPT_FGMRES_Z32, KP_OPT_OPERATOR_COLS = 1, 2, 3, 4
KP_OPT_LEARNED_GUARD, KP_OPT_SPLIT_AXIS, KP_OPT_APPLY_SMALL3 = 5, 6, 7
ELEM_LANCZOS_NOCONV, ELEM_SINGULAR_FACTOR, ELEM_SCHUR_NOCONV, ELEM_NONFINITE = 1, 2, 4, 8
ELEM_LEARNED_REJECTED, ELEM_LEARNED_WARM = 16, 32
REC_LEN = 16
PREC = {"fp64": KP_FP64, "fp32": KP_FP32, "bf16": KP_BF16, "bf16x3": KP_BF16X3}


class KpError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} (status {status})")
        self.status = status


class kp_batch(ctypes.Structure):
    _fields_ = [("num_elems", ctypes.c_int64), ("dim", ctypes.c_int32), ("n", ctypes.c_int32),
                ("params", ctypes.c_void_p), ("blocks", ctypes.c_void_p), ("nbr", ctypes.c_void_p)]


class kp_sys_batch(ctypes.Structure):
    _fields_ = [("num_elems", ctypes.c_int64), ("nc", ctypes.c_int32), ("n", ctypes.c_int32),
                ("blocks", ctypes.c_void_p)]


class kp_quad_batch(ctypes.Structure):
    _fields_ = [("num_elems", ctypes.c_int64), ("dim", ctypes.c_int32), ("n", ctypes.c_int32),
                ("mu", ctypes.c_int32), ("pad", ctypes.c_int32), ("tau", ctypes.c_double),
                ("c", ctypes.c_void_p), ("a", ctypes.c_void_p), ("nu", ctypes.c_void_p), ("g", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libkp.so (built by paper_1704_04549_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libkp.so not built ({LIB_PATH}); run paper_1704_04549_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        bp = ctypes.POINTER(kp_batch)
        sig = {
            "kp_create": ([ctypes.POINTER(vp), ctypes.c_int, vp], ctypes.c_int),
            "kp_destroy": ([vp], ctypes.c_int),
            "kp_set_stream": ([vp, vp], ctypes.c_int),
            "kp_status_string": ([ctypes.c_int], ctypes.c_char_p),
            "kp_precond_bytes": ([i32, i32, i32, i64], ctypes.c_size_t),
            "kp_build_blocks": ([vp, bp, vp], ctypes.c_int),
            "kp_setup": ([vp, bp, i32, i32, vp, vp], ctypes.c_int),
            "kp_setup_noalloc": ([vp, bp, i32, vp, vp], ctypes.c_int),
            "kp_learned_judge": ([vp, bp, i32, vp, vp, dbl, dbl, vp, vp], ctypes.c_int),
            "kp_get_axes": ([vp, bp, i32, vp, vp], ctypes.c_int),
            "kp_setup_quad": ([vp, ctypes.POINTER(kp_quad_batch), vp, vp], ctypes.c_int),
            "kp_sys_precond_bytes": ([i32, i32, i64], ctypes.c_size_t),
            "kp_setup_sys": ([vp, ctypes.POINTER(kp_sys_batch), vp, vp], ctypes.c_int),
            "kp_apply_sys": ([vp, ctypes.POINTER(kp_sys_batch), vp, i32, i32, vp, vp], ctypes.c_int),
            "kp_get_factors_sys": ([vp, ctypes.POINTER(kp_sys_batch), vp, vp, vp], ctypes.c_int),
            "kp_build_sys_blocks": ([vp, i64, i32, i32, vp, vp], ctypes.c_int),
            "kp_sys_operator_apply": ([vp, ctypes.POINTER(kp_sys_batch), vp, vp], ctypes.c_int),
            "kp_sys_blockjacobi_exact": ([vp, ctypes.POINTER(kp_sys_batch), vp, vp, vp], ctypes.c_int),
            "kp_fgmres_sys": ([vp, ctypes.POINTER(kp_sys_batch), i32, vp, vp, i32, vp, vp, i32, dbl, i32,
                               ctypes.POINTER(i32), ctypes.POINTER(dbl)], ctypes.c_int),
            "kp_setup_from_factors": ([vp, bp, i32, vp, vp, vp], ctypes.c_int),
            "kp_get_factors": ([vp, bp, i32, vp, vp, vp], ctypes.c_int),
            "kp_apply": ([vp, bp, i32, vp, i32, i32, vp, vp], ctypes.c_int),
            "kp_apply_z32": ([vp, bp, i32, vp, i32, i32, vp, vp], ctypes.c_int),
            "kp_blockjacobi_exact": ([vp, bp, vp, vp, vp], ctypes.c_int),
            "kp_blockjacobi_solve": ([vp, bp, vp, vp, i32, vp, vp], ctypes.c_int),
            "kp_operator_apply": ([vp, bp, vp, vp], ctypes.c_int),
            "kp_fgmres": ([vp, bp, i32, i32, vp, vp, i32, vp, vp, i32, dbl, i32,
                           ctypes.POINTER(i32), ctypes.POINTER(dbl), vp, i32], ctypes.c_int),
            "kp_mlp_bytes": ([i32, i32, i32], ctypes.c_size_t),
            "kp_mlp_init": ([vp, vp, i32, i32, i32, vp], ctypes.c_int),
            "kp_mlp_get": ([vp, vp, vp, vp, vp, vp], ctypes.c_int),
            "kp_mlp_set_norm": ([vp, vp, vp, vp, vp], ctypes.c_int),
            "kp_mlp_forward": ([vp, vp, i32, i64, vp, vp], ctypes.c_int),
            "kp_mlp_loss_grad": ([vp, vp, i32, i64, vp, vp, vp, vp], ctypes.c_int),
            "kp_mlp_train": ([vp, vp, bp, vp, i32, i32, ctypes.c_float, ctypes.c_uint64, i32, vp],
                             ctypes.c_int),
            "kp_mlp_predict": ([vp, vp, bp, i32, vp], ctypes.c_int),
            "kp_set_model": ([vp, vp], ctypes.c_int),
            "kp_set_option": ([vp, i32, i64], ctypes.c_int),
            "kp_mixed_plan_create": ([vp, i64, vp, ctypes.POINTER(vp)], ctypes.c_int),
            "kp_mixed_plan_destroy": ([vp], ctypes.c_int),
            "kp_mixed_plan_info": ([vp, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
            "kp_mixed_setup": ([vp, vp, vp, vp, vp], ctypes.c_int),
            "kp_mixed_get_factors": ([vp, vp, vp, vp, vp], ctypes.c_int),
            "kp_mixed_apply": ([vp, vp, vp, i32, vp, vp], ctypes.c_int),
            "kp_mixed_autotune": ([vp, vp, vp, i32, vp, vp, vp, i32], ctypes.c_int),
            "kp_mixed_operator_apply": ([vp, vp, vp, vp, vp], ctypes.c_int),
            "kp_mixed_fgmres": ([vp, vp, vp, i32, vp, i32, vp, vp, i32, dbl, i32,
                                 ctypes.POINTER(i32), ctypes.POINTER(dbl), vp, i32], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().kp_status_string(int(status)).decode()


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if t.device.type != "cuda":
            raise ValueError("device tensor expected")
        if not t.is_contiguous():
            raise ValueError("contiguous tensor expected")
        return ctypes.c_void_p(t.data_ptr())
    return t


def _check(status, what):
    if status != KP_OK:
        raise KpError(status, what)


class Batch:
    """A uniform batch (one dim, one n); holds references to its tensors."""

    def __init__(self, params: torch.Tensor, dim: int, n: int, blocks=None, nbr=None):
        if params.dtype != torch.float64 or params.shape[-1] != REC_LEN:
            raise ValueError("params must be float64 [E, 16]")
        self.params, self.blocks, self.nbr = params, blocks, nbr
        self.dim, self.n = int(dim), int(n)
        self.num_elems = int(params.shape[0])
        self.c = kp_batch(self.num_elems, self.dim, self.n, _ptr(params).value,
                          _ptr(blocks).value if blocks is not None else None,
                          _ptr(nbr).value if nbr is not None else None)

    @property
    def ndof(self) -> int:
        return self.n ** self.dim

    def nf(self, rank: int) -> int:
        return 2 * rank if self.dim == 2 else 5


class SysBatch:
    """A batch of explicit 2D blocks of nc-component systems (kp_sys_batch):
    blocks [E, nc n^2, nc n^2] float64, order (component, x, y); holds a
    reference to its tensor (None for apply-only use)."""

    def __init__(self, nc: int, n: int, blocks=None, num_elems=None):
        if blocks is not None:
            if blocks.dtype != torch.float64 or not blocks.is_contiguous():
                raise ValueError("blocks must be contiguous float64")
            num_elems = int(blocks.shape[0])
        self.nc, self.n, self.num_elems = int(nc), int(n), int(num_elems)
        self.blocks = blocks
        self.c = kp_sys_batch(self.num_elems, self.nc, self.n, _ptr(blocks).value if blocks is not None else None)

    @property
    def ndof(self) -> int:
        return self.nc * self.n * self.n


class QuadBatch:
    """A batch of general elements (kp_quad_batch): coefficients at mu points
    per axis; holds references to its tensors."""

    def __init__(self, dim: int, n: int, mu: int, tau: float, c, a, nu, g):
        for t in (c, a, nu, g):
            if t.dtype != torch.float64 or not t.is_contiguous():
                raise ValueError("quadrature data must be contiguous float64")
        self.dim, self.n, self.mu = int(dim), int(n), int(mu)
        self.num_elems = int(c.shape[0])
        self._keep = (c, a, nu, g)
        self.c = kp_quad_batch(self.num_elems, self.dim, self.n, self.mu, 0, float(tau), _ptr(c).value,
                               _ptr(a).value, _ptr(nu).value, _ptr(g).value)

    def batch(self):
        """The uniform batch (no records) that kp_apply / kp_fgmres take for it."""
        b = Batch.__new__(Batch)
        b.params = b.blocks = b.nbr = None
        b.dim, b.n, b.num_elems = self.dim, self.n, self.num_elems
        b.c = kp_batch(self.num_elems, self.dim, self.n, None, None, None)
        return b


class Ctx:
    """kp_ctx bound to a device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib().kp_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream)), "kp_create")
        self.h = h

    def close(self):
        if self.h:
            lib().kp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, option, value):
        _check(lib().kp_set_option(self.h, int(option), int(value)), "kp_set_option")

    def set_stream(self, stream):
        self.stream = stream
        _check(lib().kp_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)), "kp_set_stream")

    # ---- entry points (C names without the prefix) ----
    def precond_bytes(self, dim, n, rank, num_elems):
        return int(lib().kp_precond_bytes(dim, n, rank, num_elems))

    def build_blocks(self, b: Batch, out=None):
        N = b.ndof
        if out is None:
            out = torch.empty((b.num_elems, N, N), dtype=torch.float64, device=self.device)
        _check(lib().kp_build_blocks(self.h, ctypes.byref(b.c), _ptr(out)), "kp_build_blocks")
        return out

    def setup(self, b: Batch, rank: int = 2, mode: int = KP_SETUP_SVD, precond=None, status=None):
        if self.precond_bytes(b.dim, b.n, rank, 1) == 0:
            raise KpError(KP_ERR_ARG, "kp_precond_bytes")
        nbytes = max(self.precond_bytes(b.dim, b.n, rank, b.num_elems), 1)
        if precond is None:
            precond = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if status is None:
            status = torch.empty(b.num_elems, dtype=torch.int32, device=self.device)
        _check(lib().kp_setup(self.h, ctypes.byref(b.c), rank, mode, _ptr(precond), _ptr(status)),
               "kp_setup")
        return precond, status

    def setup_noalloc(self, b: Batch, rank: int, precond: torch.Tensor, status: torch.Tensor = None):
        """kp_setup_noalloc: the caller passes the preconditioner buffer (and the
        status array, or None); the library allocates nothing."""
        _check(lib().kp_setup_noalloc(self.h, ctypes.byref(b.c), rank, _ptr(precond), _ptr(status)),
               "kp_setup_noalloc")
        return precond, status

    def learned_judge(self, b: Batch, pred_factors: torch.Tensor, precond, factor=1.1, guard=0.1):
        """kp_learned_judge (rank 2): returns (out [E][4], accept [E])."""
        out = torch.empty((b.num_elems, 4), dtype=torch.float64, device=self.device)
        acc = torch.empty(b.num_elems, dtype=torch.int32, device=self.device)
        _check(lib().kp_learned_judge(self.h, ctypes.byref(b.c), 2, _ptr(pred_factors), _ptr(precond),
                                      float(factor), float(guard), _ptr(out), _ptr(acc)), "kp_learned_judge")
        return out, acc

    def setup_quad(self, q: QuadBatch, precond=None, status=None):
        nbytes = max(self.precond_bytes(q.dim, q.n, 2, q.num_elems), 1)
        if precond is None:
            precond = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if status is None:
            status = torch.empty(q.num_elems, dtype=torch.int32, device=self.device)
        _check(lib().kp_setup_quad(self.h, ctypes.byref(q.c), _ptr(precond), _ptr(status)), "kp_setup_quad")
        return precond, status

    def sys_precond_bytes(self, nc: int, n: int, num_elems: int) -> int:
        return int(lib().kp_sys_precond_bytes(int(nc), int(n), int(num_elems)))

    def setup_sys(self, s: "SysBatch", precond=None, status=None):
        nbytes = self.sys_precond_bytes(s.nc, s.n, s.num_elems)
        if nbytes == 0 and s.num_elems > 0:
            raise KpError(KP_ERR_ARG, "kp_sys_precond_bytes")
        if precond is None:
            precond = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self.device)
        if status is None:
            status = torch.empty(max(s.num_elems, 1), dtype=torch.int32, device=self.device)
        _check(lib().kp_setup_sys(self.h, ctypes.byref(s.c), _ptr(precond), _ptr(status)), "kp_setup_sys")
        return precond, status

    def apply_sys(self, s: "SysBatch", precond, prec, r: torch.Tensor, z=None):
        prec = PREC.get(prec, prec)
        if r.dtype != torch.float64:
            raise ValueError("r must be float64")
        nrhs = r.numel() // (s.num_elems * s.ndof) if s.num_elems else 1
        if z is None:
            z = torch.empty_like(r)
        _check(lib().kp_apply_sys(self.h, ctypes.byref(s.c), _ptr(precond), int(prec), int(nrhs), _ptr(r),
                                  _ptr(z)), "kp_apply_sys")
        return z

    def get_factors_sys(self, s: "SysBatch", precond):
        m, n = s.nc * s.n, s.n
        f = torch.empty((s.num_elems, 2 * m * m + 2 * n * n), dtype=torch.float64, device=self.device)
        sg = torch.empty((s.num_elems, 4), dtype=torch.float64, device=self.device)
        _check(lib().kp_get_factors_sys(self.h, ctypes.byref(s.c), _ptr(precond), _ptr(f), _ptr(sg)),
               "kp_get_factors_sys")
        return f, sg

    def build_sys_blocks(self, nc: int, n: int, recs: torch.Tensor, out=None):
        E = int(recs.shape[0]) if recs.numel() else 0
        N = nc * n * n
        if out is None:
            out = torch.empty((E, N, N), dtype=torch.float64, device=self.device)
        _check(lib().kp_build_sys_blocks(self.h, E, int(nc), int(n), _ptr(recs), _ptr(out)), "kp_build_sys_blocks")
        return out

    def sys_operator_apply(self, s: "SysBatch", x, y=None):
        if y is None:
            y = torch.empty_like(x)
        _check(lib().kp_sys_operator_apply(self.h, ctypes.byref(s.c), _ptr(x), _ptr(y)), "kp_sys_operator_apply")
        return y

    def sys_blockjacobi_exact(self, s: "SysBatch", lu=None, piv=None, status=None):
        N = s.ndof
        if lu is None:
            lu = torch.empty((s.num_elems, N, N), dtype=torch.float64, device=self.device)
        if piv is None:
            piv = torch.empty((s.num_elems, N), dtype=torch.int32, device=self.device)
        if status is None:
            status = torch.empty(max(s.num_elems, 1), dtype=torch.int32, device=self.device)
        _check(lib().kp_sys_blockjacobi_exact(self.h, ctypes.byref(s.c), _ptr(lu), _ptr(piv), _ptr(status)),
               "kp_sys_blockjacobi_exact")
        return lu, piv, status

    def fgmres_sys(self, s: "SysBatch", rhs, pc_kind=KP_PC_KSVD, pc_data=None, pc_aux=None, pc_prec=KP_FP64,
                   x=None, restart=30, rtol=1e-10, maxit=3000):
        pc_prec = PREC.get(pc_prec, pc_prec)
        if x is None:
            x = torch.empty_like(rhs)
        it = ctypes.c_int32(0)
        rr = ctypes.c_double(0.0)
        st = lib().kp_fgmres_sys(self.h, ctypes.byref(s.c), int(pc_kind), _ptr(pc_data), _ptr(pc_aux), int(pc_prec),
                                 _ptr(rhs), _ptr(x), int(restart), float(rtol), int(maxit), ctypes.byref(it),
                                 ctypes.byref(rr))
        if st not in (KP_OK, KP_ERR_NOCONV):
            raise KpError(st, "kp_fgmres_sys")
        return dict(x=x, iters=it.value, relres=rr.value, converged=(st == KP_OK))

    def setup_from_factors(self, b: Batch, rank: int, factors: torch.Tensor, precond=None, status=None):
        if self.precond_bytes(b.dim, b.n, rank, 1) == 0:
            raise KpError(KP_ERR_ARG, "kp_precond_bytes")
        nbytes = max(self.precond_bytes(b.dim, b.n, rank, b.num_elems), 1)
        if precond is None:
            precond = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if status is None:
            status = torch.empty(b.num_elems, dtype=torch.int32, device=self.device)
        _check(lib().kp_setup_from_factors(self.h, ctypes.byref(b.c), rank, _ptr(factors),
                                           _ptr(precond), _ptr(status)), "kp_setup_from_factors")
        return precond, status

    def get_factors(self, b: Batch, rank: int, precond):
        f = torch.empty((b.num_elems, b.nf(rank), b.n, b.n), dtype=torch.float64, device=self.device)
        s = torch.empty((b.num_elems, 4), dtype=torch.float64, device=self.device)
        _check(lib().kp_get_factors(self.h, ctypes.byref(b.c), rank, _ptr(precond), _ptr(f), _ptr(s)),
               "kp_get_factors")
        return f, s

    def get_axes(self, b: Batch, rank: int, precond):
        ax = torch.empty(b.num_elems, dtype=torch.int8, device=self.device)
        _check(lib().kp_get_axes(self.h, ctypes.byref(b.c), rank, _ptr(precond), _ptr(ax)), "kp_get_axes")
        return ax

    def apply(self, b: Batch, rank: int, precond, prec, r: torch.Tensor, z=None):
        prec = PREC.get(prec, prec)
        if r.dtype != torch.float64:
            raise ValueError("r must be float64")
        nrhs = r.numel() // (b.num_elems * b.ndof) if b.num_elems else 1
        if z is None:
            z = torch.empty_like(r)
        _check(lib().kp_apply(self.h, ctypes.byref(b.c), rank, _ptr(precond), int(prec), int(nrhs),
                              _ptr(r), _ptr(z)), "kp_apply")
        return z

    def apply_z32(self, b: Batch, rank: int, precond, prec, r: torch.Tensor, z=None):
        """kp_apply_z32: as apply, z float32 (rank 2; prec fp32, bf16 or bf16x3)."""
        prec = PREC.get(prec, prec)
        if r.dtype != torch.float64:
            raise ValueError("r must be float64")
        nrhs = r.numel() // (b.num_elems * b.ndof) if b.num_elems else 1
        if z is None:
            z = torch.empty(r.shape, dtype=torch.float32, device=r.device)
        if z.dtype != torch.float32 or z.numel() != r.numel():
            raise ValueError("z must be float32 with r's size")
        _check(lib().kp_apply_z32(self.h, ctypes.byref(b.c), rank, _ptr(precond), int(prec), int(nrhs),
                                  _ptr(r), _ptr(z)), "kp_apply_z32")
        return z

    def blockjacobi_exact(self, b: Batch, lu=None, piv=None, status=None):
        N = b.ndof
        if lu is None:
            lu = torch.empty((b.num_elems, N, N), dtype=torch.float64, device=self.device)
        if piv is None:
            piv = torch.empty((b.num_elems, N), dtype=torch.int32, device=self.device)
        if status is None:
            status = torch.empty(b.num_elems, dtype=torch.int32, device=self.device)
        _check(lib().kp_blockjacobi_exact(self.h, ctypes.byref(b.c), _ptr(lu), _ptr(piv), _ptr(status)),
               "kp_blockjacobi_exact")
        return lu, piv, status

    def blockjacobi_solve(self, b: Batch, lu, piv, r, z=None):
        nrhs = r.numel() // (b.num_elems * b.ndof) if b.num_elems else 1
        if z is None:
            z = torch.empty_like(r)
        _check(lib().kp_blockjacobi_solve(self.h, ctypes.byref(b.c), _ptr(lu), _ptr(piv), int(nrhs),
                                          _ptr(r), _ptr(z)), "kp_blockjacobi_solve")
        return z

    def operator_apply(self, b: Batch, x, y=None):
        if y is None:
            y = torch.empty_like(x)
        _check(lib().kp_operator_apply(self.h, ctypes.byref(b.c), _ptr(x), _ptr(y)), "kp_operator_apply")
        return y

    def fgmres(self, b: Batch, rhs, pc_kind=KP_PC_KSVD, rank=2, pc_data=None, pc_aux=None,
               pc_prec=KP_FP64, x=None, restart=30, rtol=1e-10, maxit=3000, hist_len=0):
        pc_prec = PREC.get(pc_prec, pc_prec)
        if x is None:
            x = torch.empty_like(rhs)
        it = ctypes.c_int32(0)
        rr = ctypes.c_double(0.0)
        hist = (ctypes.c_double * max(hist_len, 1))()
        st = lib().kp_fgmres(self.h, ctypes.byref(b.c), int(pc_kind), int(rank), _ptr(pc_data),
                             _ptr(pc_aux), int(pc_prec), _ptr(rhs), _ptr(x), int(restart), float(rtol), int(maxit),
                             ctypes.byref(it), ctypes.byref(rr), hist if hist_len > 0 else None,
                             int(hist_len))
        if st not in (KP_OK, KP_ERR_NOCONV):
            raise KpError(st, "kp_fgmres")
        return dict(x=x, iters=it.value, relres=rr.value, converged=(st == KP_OK),
                    hist=list(hist)[:min(hist_len, it.value)])

    # ------------------------------------------------------ learned setup
    def mlp_param_count(self, dim, n, hidden):
        O = (5 if dim == 3 else 4) * n * n
        return hidden * 12 + hidden + hidden * hidden + hidden + O * hidden + O

    def mlp_create(self, dim, n, hidden, params=None):
        """A model buffer initialised with params (FP32 device tensor of P values) or zeros."""
        nbytes = int(lib().kp_mlp_bytes(dim, n, hidden))
        if nbytes == 0:
            raise KpError(KP_ERR_ARG, "kp_mlp_bytes")
        model = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if params is not None and (params.dtype != torch.float32 or
                                   params.numel() != self.mlp_param_count(dim, n, hidden)):
            raise ValueError("params: float32 tensor of the model's parameter count expected")
        _check(lib().kp_mlp_init(self.h, _ptr(model), dim, n, hidden, _ptr(params)), "kp_mlp_init")
        return model

    def mlp_get(self, model, dim, n, hidden):
        P = self.mlp_param_count(dim, n, hidden)
        params = torch.empty(P, dtype=torch.float32, device=self.device)
        xm = torch.empty(12, dtype=torch.float32, device=self.device)
        xs = torch.empty(12, dtype=torch.float32, device=self.device)
        ys = torch.empty(5 if dim == 3 else 4, dtype=torch.float32, device=self.device)
        _check(lib().kp_mlp_get(self.h, _ptr(model), _ptr(params), _ptr(xm), _ptr(xs), _ptr(ys)), "kp_mlp_get")
        return params, xm, xs, ys

    def mlp_set_norm(self, model, x_mean=None, x_std=None, yscale=None):
        _check(lib().kp_mlp_set_norm(self.h, _ptr(model), _ptr(x_mean), _ptr(x_std), _ptr(yscale)),
               "kp_mlp_set_norm")

    def mlp_forward(self, model, xn, out_dim, prec="fp32"):
        prec = PREC.get(prec, prec)
        y = torch.empty((xn.shape[0], out_dim), dtype=torch.float32, device=self.device)
        _check(lib().kp_mlp_forward(self.h, _ptr(model), int(prec), int(xn.shape[0]), _ptr(xn), _ptr(y)),
               "kp_mlp_forward")
        return y

    def mlp_loss_grad(self, model, xn, t, n_params, prec="fp32"):
        prec = PREC.get(prec, prec)
        g = torch.empty(n_params, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _check(lib().kp_mlp_loss_grad(self.h, _ptr(model), int(prec), int(xn.shape[0]), _ptr(xn), _ptr(t),
                                      _ptr(g), _ptr(loss)), "kp_mlp_loss_grad")
        return loss, g

    def mlp_train(self, model, b: Batch, factors, epochs, batch=256, lr=1e-3, seed=3004, prec="fp32"):
        prec = PREC.get(prec, prec)
        hist = (ctypes.c_float * max(epochs, 1))()
        _check(lib().kp_mlp_train(self.h, _ptr(model), ctypes.byref(b.c), _ptr(factors), int(epochs),
                                  int(batch), float(lr), int(seed), int(prec), hist), "kp_mlp_train")
        return list(hist)[:epochs]

    def mlp_predict(self, model, b: Batch, prec="fp32"):
        prec = PREC.get(prec, prec)
        f = torch.empty((b.num_elems, 5 if b.dim == 3 else 4, b.n, b.n), dtype=torch.float64,
                        device=self.device)
        _check(lib().kp_mlp_predict(self.h, _ptr(model), ctypes.byref(b.c), int(prec), _ptr(f)),
               "kp_mlp_predict")
        return f

    def set_model(self, model):
        _check(lib().kp_set_model(self.h, _ptr(model)), "kp_set_model")


class MixedPlan:
    """A mixed batch (per-element dim and n) and its plan; records on the device."""

    def __init__(self, ctx: "Ctx", dims, ns, params: torch.Tensor):
        import numpy as np
        self.ctx = ctx
        self.dims = np.asarray(dims, dtype=np.int32)
        self.ns = np.asarray(ns, dtype=np.int32)
        self.E = int(self.dims.size)
        if params.dtype != torch.float64 or tuple(params.shape) != (self.E, REC_LEN):
            raise ValueError("params: float64 [E, 16] device tensor expected")
        self.params = params
        dn = np.ascontiguousarray(np.stack([self.dims, self.ns], axis=1).astype(np.int32))
        h = ctypes.c_void_p()
        _check(lib().kp_mixed_plan_create(ctx.h, self.E, dn.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)),
               "kp_mixed_plan_create")
        self.h = h
        vl = ctypes.c_int64(0)
        pb = ctypes.c_size_t(0)
        _check(lib().kp_mixed_plan_info(self.h, ctypes.byref(vl), ctypes.byref(pb)), "kp_mixed_plan_info")
        self.vec_len = vl.value
        self.precond_bytes = pb.value
        offs = np.zeros(self.E + 1, dtype=np.int64)
        offs[1:] = np.cumsum(self.ns.astype(np.int64) ** self.dims)
        self.offsets = offs

    def close(self):
        if self.h:
            lib().kp_mixed_plan_destroy(self.h)
            self.h = None

    def setup(self, precond=None, status=None):
        if precond is None:
            precond = torch.empty(max(self.precond_bytes, 1), dtype=torch.uint8, device=self.ctx.device)
        if status is None:
            status = torch.empty(self.E, dtype=torch.int32, device=self.ctx.device)
        _check(lib().kp_mixed_setup(self.ctx.h, self.h, _ptr(self.params), _ptr(precond), _ptr(status)),
               "kp_mixed_setup")
        return precond, status

    def get_factors(self, precond):
        import numpy as np
        total = int(np.sum(np.where(self.dims == 3, 5, 4) * self.ns.astype(np.int64) ** 2))
        f = torch.empty(total, dtype=torch.float64, device=self.ctx.device)
        sg = torch.empty((self.E, 4), dtype=torch.float64, device=self.ctx.device)
        _check(lib().kp_mixed_get_factors(self.ctx.h, self.h, _ptr(precond), _ptr(f), _ptr(sg)),
               "kp_mixed_get_factors")
        return f, sg

    def apply(self, precond, prec, r, z=None):
        prec = PREC.get(prec, prec)
        if z is None:
            z = torch.empty_like(r)
        _check(lib().kp_mixed_apply(self.ctx.h, self.h, _ptr(precond), int(prec), _ptr(r), _ptr(z)),
               "kp_mixed_apply")
        return z

    def autotune(self, precond, prec, r, z):
        prec = PREC.get(prec, prec)
        buf = (ctypes.c_int32 * 300)()
        _check(lib().kp_mixed_autotune(self.ctx.h, self.h, _ptr(precond), int(prec), _ptr(r), _ptr(z), buf, 300),
               "kp_mixed_autotune")
        out = {}
        for i in range(0, 300, 3):
            if buf[i] < 0:
                break
            out[(buf[i], buf[i + 1])] = buf[i + 2]
        return out

    def operator_apply(self, x, y=None):
        if y is None:
            y = torch.empty_like(x)
        _check(lib().kp_mixed_operator_apply(self.ctx.h, self.h, _ptr(self.params), _ptr(x), _ptr(y)),
               "kp_mixed_operator_apply")
        return y

    def fgmres(self, rhs, pc_kind=KP_PC_KSVD, precond=None, pc_prec=KP_FP64, x=None, restart=30, rtol=1e-10,
               maxit=3000):
        pc_prec = PREC.get(pc_prec, pc_prec)
        if x is None:
            x = torch.empty_like(rhs)
        it = ctypes.c_int32(0)
        rr = ctypes.c_double(0.0)
        st = lib().kp_mixed_fgmres(self.ctx.h, self.h, _ptr(self.params), int(pc_kind), _ptr(precond),
                                   int(pc_prec), _ptr(rhs), _ptr(x), int(restart), float(rtol), int(maxit),
                                   ctypes.byref(it), ctypes.byref(rr), None, 0)
        if st not in (KP_OK, KP_ERR_NOCONV):
            raise KpError(st, "kp_mixed_fgmres")
        return dict(x=x, iters=it.value, relres=rr.value, converged=(st == KP_OK))
