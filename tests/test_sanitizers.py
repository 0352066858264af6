"""The FP64 oracles under AddressSanitizer and UndefinedBehaviorSanitizer:
both C sources built with the sanitizers (oracle.build(sanitize=True)) and
loaded, through IJ_ORACLE_LIB / IJ_ORACLE3D_LIB, by a child pytest that runs
the oracles' pin tests (every step, diagnostic and boundary path they reach)
with the sanitizer runtime preloaded.  Any sanitizer report fails."""
import os
import subprocess
import sys

import pytest

from oracle import oracle as O
from oracle import oracle3d as O3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_oracles_under_sanitizers(tmp_path):
    asan = _runtime()
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    lib2 = O.build(out=str(tmp_path / "liblbm_oracle_san.so"), sanitize=True)
    lib3 = O3.build(out=str(tmp_path / "liblbm3d_oracle_san.so"), sanitize=True)
    env = dict(os.environ, LD_PRELOAD=asan, IJ_ORACLE_LIB=lib2, IJ_ORACLE3D_LIB=lib3,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               OMP_NUM_THREADS="4")
    # the Laplace-law and wide contact-angle runs repeat the code paths of the
    # others over many more steps: left out for time
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
           "-k", "not wide and not laplace", "tests/test_oracle_pins.py", "tests/test_oracle3d_pins.py", "tests/test_oracle_diag.py",
           "tests/test_golden.py"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert " passed" in out
