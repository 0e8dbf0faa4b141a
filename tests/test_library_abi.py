"""The C-ABI library loads and exports every symbol include/kp.h declares (no GPU needed)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "kp.h")).read()
    return sorted(set(re.findall(r"^\s*(?:kp_status|size_t|const char\*)\s+(kp_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("kp_setup", "kp_apply", "kp_blockjacobi_exact", "kp_fgmres", "kp_operator_apply"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1704_04549_amd", "libkp.so"))
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_precond_bytes_and_status_strings():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1704_04549_amd", "libkp.so"))
    lib.kp_precond_bytes.restype = ctypes.c_size_t
    lib.kp_precond_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64]
    assert lib.kp_precond_bytes(3, 16, 2, 10) > 10 * (7 + 16) * 256 * 8
    assert lib.kp_precond_bytes(3, 16, 1, 10) == 0   # 3D has the two-stage rank-2 form only
    assert lib.kp_precond_bytes(2, 33, 2, 10) == 0   # n above 32
    assert lib.kp_precond_bytes(4, 8, 2, 10) == 0
    lib.kp_status_string.restype = ctypes.c_char_p
    assert lib.kp_status_string(0) == b"ok"
    assert lib.kp_status_string(1) == b"invalid argument"
