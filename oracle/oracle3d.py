"""ctypes wrapper around the FP64 CPU oracle of the three-dimensional update
(``lbm3d_oracle.c``: D3Q19 f, D3Q7 g, the readings of the two-dimensional
oracle carried to three dimensions).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline of the benchmark use this module; the GPU library never imports it,
and this module imports nothing from the GPU library.

Arrays are indexed ``[y, z, x]`` (x fastest); ``wall`` is ``uint8`` with
0 fluid, 1 inner nozzle wall, 2 outer plate.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm3d_oracle.c")
LIB = os.path.join(HERE, "liblbm3d_oracle.so")


# Flags of the sanitizer build (AddressSanitizer and UndefinedBehaviorSanitizer)
SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


def build(force: bool = True, out: Optional[str] = None, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, no contraction of a*b+c).

    With `sanitize`: the same source built with SANITIZE instead of -O2
    into `out`, the library that the test-suite's sanitizer run loads
    through the IJ_ORACLE3D_LIB environment variable."""
    target = out or LIB
    if sanitize or force or not os.path.exists(target) or os.path.getmtime(target) < os.path.getmtime(SRC):
        tmp = target + ".tmp"
        opt = SANITIZE if sanitize else ["-O2"]
        subprocess.check_call(["gcc", *opt, "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp",
                               "-ffp-contract=off", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, target)
    return target


class _Params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("nx", "ny", "nz", "bc_y", "force_rows", "t_pos", "t_neg", "t_idle", "periodic_pulse")] + \
               [(k, ctypes.c_double) for k in
                ("rho_ink", "rho_amb", "sigma", "width", "gamma", "tau_ink", "tau_amb", "tau_phi",
                 "theta_inner", "theta_outer", "f_pos", "f_neg")]


PARAM_KEYS = [name for name, _ in _Params._fields_]
Q, QG = 19, 7
_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("IJ_ORACLE3D_LIB") or LIB
        if path == LIB and not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(path)
        vp = ctypes.c_void_p
        L.o3_create.restype = vp
        L.o3_create.argtypes = [ctypes.POINTER(_Params), vp, ctypes.POINTER(ctypes.c_int)]
        L.o3_destroy.argtypes = [vp]
        L.o3_derived.argtypes = [vp, vp]
        L.o3_velocity_set.argtypes = [vp, vp, vp]
        L.o3_init_phi.argtypes = [vp] * 5
        L.o3_step.argtypes = [vp, ctypes.c_long]
        L.o3_time.argtypes = [vp]
        L.o3_time.restype = ctypes.c_long
        L.o3_fields.argtypes = [vp] * 8
        L.o3_get_state.argtypes = [vp, vp, vp]
        L.o3_set_state.argtypes = [vp, vp, vp, ctypes.c_long]
        L.o3_diag.argtypes = [vp, ctypes.c_long, vp, vp, vp]
        L.o3_pulse.restype = ctypes.c_double
        L.o3_pulse.argtypes = [ctypes.POINTER(_Params), ctypes.c_long]
        L.o3_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _params(p: dict) -> _Params:
    return _Params(**{k: p[k] for k in PARAM_KEYS})


def set_threads(n: int) -> None:
    lib().o3_set_threads(int(n))


def velocity_set():
    """(c[19, 3], w[19], opp[19]) of the oracle's D3Q19 set."""
    c = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q)
    opp = np.zeros(Q, dtype=np.int32)
    lib().o3_velocity_set(_ptr(c), _ptr(w), _ptr(opp))
    return c, w, opp


class Oracle3D:
    """FP64 three-dimensional simulation on the CPU."""

    def __init__(self, params: dict, wall: np.ndarray):
        self.p = dict(params)
        ny, nz, nx = int(params["ny"]), int(params["nz"]), int(params["nx"])
        self.shape = (ny, nz, nx)
        w = np.ascontiguousarray(wall, dtype=np.uint8)
        assert w.shape == self.shape, (w.shape, self.shape)
        self.wall = w
        self._pp = _params(params)
        err = ctypes.c_int(0)
        self.h = lib().o3_create(ctypes.byref(self._pp), _ptr(w), ctypes.byref(err))
        if not self.h:
            raise ValueError(f"o3_create failed (code {err.value})")

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.o3_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def derived(self) -> dict:
        out = np.zeros(7)
        lib().o3_derived(self.h, _ptr(out))
        return dict(zip(("phi_star", "n0", "beta", "kappa", "q", "wet_inner", "wet_outer"), out))

    def init_phi(self, phi, ux=None, uy=None, uz=None):
        c = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(self.shape)
        phi, ux, uy, uz = c(phi), c(ux), c(uy), c(uz)
        lib().o3_init_phi(self.h, _ptr(phi), _ptr(ux), _ptr(uy), _ptr(uz))

    def init_distance(self, d):
        ps = self.derived()["phi_star"]
        self.init_phi(ps * np.tanh(2.0 * np.asarray(d, dtype=np.float64) / self.p["width"]))

    def step(self, n: int = 1):
        lib().o3_step(self.h, int(n))

    @property
    def t(self) -> int:
        return lib().o3_time(self.h)

    def fields(self) -> dict:
        out = {k: np.zeros(self.shape) for k in ("n", "phi", "ux", "uy", "uz", "phi_tilde", "mu")}
        lib().o3_fields(self.h, *(_ptr(out[k]) for k in ("n", "phi", "ux", "uy", "uz", "phi_tilde", "mu")))
        return out

    def get_state(self):
        f = np.zeros((Q,) + self.shape)
        g = np.zeros((QG,) + self.shape)
        lib().o3_get_state(self.h, _ptr(f), _ptr(g))
        return f, g

    def set_state(self, f, g, t: int = 0):
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        assert f.shape == (Q,) + self.shape and g.shape == (QG,) + self.shape
        lib().o3_set_state(self.h, _ptr(f), _ptr(g), int(t))

    def diag(self, row0: int = 0) -> dict:
        rec = np.zeros(7)
        cnt = np.zeros(self.shape[0], dtype=np.int64)
        uy = np.zeros(self.shape[0])
        lib().o3_diag(self.h, int(row0), _ptr(rec), _ptr(cnt), _ptr(uy))
        return dict(mass_n=rec[0], mass_phi=rec[1], mom=rec[2:5].copy(), max_u=rec[5], nan_count=int(rec[6]),
                    row_count=cnt, row_uy=uy)
