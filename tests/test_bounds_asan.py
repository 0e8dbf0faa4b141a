"""Host builds of the per-element routines under AddressSanitizer and
UndefinedBehaviorSanitizer (tests/native/bounds_check.cpp): every array an
element's routine reads sits in a heap buffer of exactly its layout size, for
table formation and the generic apply (2D n = 2..32, 3D n = 2..16; FP64, FP32,
BF16, split BF16), the structured setup, the learned-setup judge, the
general-element setup and the systems blocks (setup, tables, apply).  CPU
only; skipped where g++ lacks the sanitizers."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1704_04549_amd", "csrc")


def test_per_element_routines_stay_in_bounds():
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not found")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "bounds_check")
        cmd = [cxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               f"-I{CSRC}", os.path.join(ROOT, "tests", "native", "bounds_check.cpp"),
               os.path.join(CSRC, "tables.cpp"), os.path.join(CSRC, "quad_tables.cpp"), "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0 and "sanitize" in r.stderr:
            pytest.skip("sanitizers unavailable: " + r.stderr[-300:])
        assert r.returncode == 0, r.stderr[-2000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
        run = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
        assert run.returncode == 0, (run.stdout[-1000:], run.stderr[-3000:])
        assert "checked" in run.stdout
