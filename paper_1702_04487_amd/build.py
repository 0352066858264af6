"""Build the HIP library (``libinkjet_lbm.so``) and the copy calibration
program (``bin/copy_calib``) in-tree for gfx950."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libinkjet_lbm.so")
SOURCES = [os.path.join(CSRC, f) for f in ("lbm_core.hip", "ij_api.cpp", "ij_batch.cpp", "mlp.hip", "ij_mlp.cpp",
                                          "lbm3d.hip")]
CALIB = os.path.join(HERE, "bin", "copy_calib")

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


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    _hipcc(["-shared", "-o", tmp, *SOURCES], verbose)
    os.replace(tmp, LIB)
    os.makedirs(os.path.dirname(CALIB), exist_ok=True)
    _hipcc(["-o", CALIB + ".tmp", os.path.join(CSRC, "copy_calib.hip")], verbose)
    os.replace(CALIB + ".tmp", CALIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
