"""Build the HIP library (``libinkjet_lbm.so``), the copy calibration
program (``bin/copy_calib``) and the C ABI exercise with its host code under
AddressSanitizer and UndefinedBehaviorSanitizer (``bin/abi_exercise_asan``,
run by the test-suite) in-tree for gfx950."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libinkjet_lbm.so")
SOURCES = [os.path.join(CSRC, f) for f in ("lbm_core.hip", "ij_api.cpp", "ij_batch.cpp", "mlp.hip", "ij_mlp.cpp",
                                          "lbm3d.hip")]
CALIB = os.path.join(HERE, "bin", "copy_calib")
EXERCISE_SRC = os.path.join(ROOT, "tests", "native", "abi_exercise.cpp")
EXERCISE = os.path.join(HERE, "bin", "abi_exercise_asan")
CLANGXX = os.environ.get("CLANGXX", "/opt/rocm/llvm/bin/clang++")
# host code only: the device code of these objects is built as usual
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# -packed-fp32-ops: no v_pk_*_f32 (their forms are avoided on this target);
# -ffp-contract=on: contraction decided per source expression, so every
# kernel that inlines the same node arithmetic rounds it the same way.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _hipcc(args, verbose):
    cmd = [HIPCC, *FLAGS, *args]
    if verbose:
        print(" ".join(cmd))
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops"
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed:\n{msg}")
    if verbose and msg.strip():
        print(msg)


def build_exercise(verbose: bool = False) -> str:
    """The library sources and tests/native/abi_exercise.cpp compiled with
    SANITIZE_HOST (one object each, in parallel), linked by clang++ with the
    sanitizer runtimes."""
    obj_dir = os.path.join(HERE, "bin", "abi_exercise_objs")
    os.makedirs(obj_dir, exist_ok=True)
    srcs = SOURCES + [EXERCISE_SRC]
    objs = [os.path.join(obj_dir, os.path.basename(f) + ".o") for f in srcs]
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        jobs = [ex.submit(_hipcc, [*SANITIZE_HOST, "-c", "-x", "hip", src, "-o", obj], verbose)
                for src, obj in zip(srcs, objs)]
        for j in jobs:
            j.result()
    link = [CLANGXX, "-fsanitize=address,undefined", "-o", EXERCISE + ".tmp", *objs,
            "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link of the sanitizer exercise failed:\n" + r.stdout + r.stderr)
    os.replace(EXERCISE + ".tmp", EXERCISE)
    return EXERCISE


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    _hipcc(["-shared", "-o", tmp, *SOURCES], verbose)
    os.replace(tmp, LIB)
    os.makedirs(os.path.dirname(CALIB), exist_ok=True)
    _hipcc(["-o", CALIB + ".tmp", os.path.join(CSRC, "copy_calib.hip")], verbose)
    os.replace(CALIB + ".tmp", CALIB)
    build_exercise(verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
