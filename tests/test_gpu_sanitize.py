"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(device code built as usual): tests/native/abi_exercise.cpp calls every entry
point of include/inkjet_lbm.h, with valid arguments and with the invalid ones
each declaration documents, in a program whose host objects carry the
sanitizers (built by paper_1702_04487_amd/build.py).  Any report of either
sanitizer, or an unexpected status, fails the test."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_1702_04487_amd", "bin", "abi_exercise_asan")


def test_c_abi_host_code_under_sanitizers(gpu_lib):
    assert os.path.exists(EXE), "build first: python -m paper_1702_04487_amd.build"
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    print("running", EXE, flush=True)
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=180, env=env)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert r.returncode == 0 and "abi_exercise: ok" in out, out[-6000:]
