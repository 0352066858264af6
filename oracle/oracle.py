"""ctypes wrapper around the FP64 CPU oracle (``lbm_oracle.c``) plus the
plain-Python post-processing of the droplet diagnostics.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline of the benchmark use this module; the GPU library never imports it,
and this module imports nothing from the GPU library.

Parameter dictionaries use the keys of :data:`PARAM_KEYS`; geometry is a
``uint8`` array ``wall[y, x]`` (0 fluid, 1 inner nozzle wall, 2 outer plate).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")


# Flags of the sanitizer build (AddressSanitizer and UndefinedBehaviorSanitizer)
SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


def build(force: bool = True, out: Optional[str] = None, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, strict IEEE double arithmetic).

    With `sanitize`: the same source built with SANITIZE instead of -O2
    into `out`, the library that the test-suite's sanitizer run loads
    through the IJ_ORACLE_LIB environment variable."""
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
                ("nx", "ny", "bc_y", "force_rows", "t_pos", "t_neg", "t_idle", "periodic_pulse")] + \
               [(k, ctypes.c_double) for k in
                ("rho_ink", "rho_amb", "sigma", "width", "gamma", "tau_ink", "tau_amb", "tau_phi",
                 "theta_inner", "theta_outer", "f_pos", "f_neg")]


PARAM_KEYS = [name for name, _ in _Params._fields_]

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("IJ_ORACLE_LIB") or LIB
        if path == LIB and not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.o_create.restype = ctypes.c_void_p
        L.o_create.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]
        L.o_destroy.argtypes = [ctypes.c_void_p]
        L.o_derived.argtypes = [ctypes.c_void_p, dp]
        L.o_init_phi.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.o_init_distance.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.o_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
        L.o_time.argtypes = [ctypes.c_void_p]
        L.o_time.restype = ctypes.c_long
        L.o_fields.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 11
        L.o_get_state.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.o_set_state.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_long]
        L.o_diag.argtypes = [ctypes.c_void_p, ctypes.c_long, dp, ctypes.c_void_p, ctypes.c_void_p]
        L.o_omega_of_theta.restype = ctypes.c_double
        L.o_omega_of_theta.argtypes = [ctypes.c_double]
        L.o_cos_theta_of_omega.restype = ctypes.c_double
        L.o_cos_theta_of_omega.argtypes = [ctypes.c_double]
        L.o_pulse.restype = ctypes.c_double
        L.o_pulse.argtypes = [ctypes.POINTER(_Params), ctypes.c_long]
        L.o_set_threads.argtypes = [ctypes.c_int]
        L.o_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _params(p: dict) -> _Params:
    s = _Params()
    for k in PARAM_KEYS:
        setattr(s, k, p[k])
    return s


def set_threads(n: int) -> None:
    lib().o_set_threads(int(n))


def max_threads() -> int:
    return int(lib().o_max_threads())


def omega_of_theta(theta_deg: float) -> float:
    return lib().o_omega_of_theta(float(theta_deg))


def cos_theta_of_omega(om: float) -> float:
    return lib().o_cos_theta_of_omega(float(om))


def pulse(p: dict, t: int) -> float:
    return lib().o_pulse(ctypes.byref(_params(p)), int(t))


class OracleSim:
    """One lattice simulated by the FP64 oracle."""

    def __init__(self, params: dict, wall: np.ndarray):
        self.p = dict(params)
        self.nx, self.ny = int(params["nx"]), int(params["ny"])
        self.wall = np.ascontiguousarray(wall, dtype=np.uint8)
        assert self.wall.shape == (self.ny, self.nx)
        err = ctypes.c_int(0)
        self._pp = _params(self.p)
        h = lib().o_create(ctypes.byref(self._pp), _ptr(self.wall), ctypes.byref(err))
        if not h:
            raise ValueError(f"oracle rejected the parameters/geometry (code {err.value})")
        self.h = ctypes.c_void_p(h)

    def close(self):
        if getattr(self, "h", None):
            lib().o_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    # ---- constants ----
    def derived(self) -> dict:
        out = np.zeros(8)
        lib().o_derived(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        keys = ["phi_star", "n0", "beta", "kappa", "q", "wet_inner", "wet_outer", "mobility"]
        return dict(zip(keys, out.tolist()))

    # ---- initial state ----
    def init_phi(self, phi, ux=None, uy=None):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        ux = None if ux is None else np.ascontiguousarray(ux, dtype=np.float64)
        uy = None if uy is None else np.ascontiguousarray(uy, dtype=np.float64)
        lib().o_init_phi(self.h, _ptr(phi), _ptr(ux), _ptr(uy))

    def init_distance(self, d):
        d = np.ascontiguousarray(d, dtype=np.float64)
        lib().o_init_distance(self.h, _ptr(d))

    # ---- stepping ----
    def step(self, n: int = 1):
        lib().o_step(self.h, int(n))

    @property
    def t(self) -> int:
        return int(lib().o_time(self.h))

    # ---- readback ----
    def fields(self) -> dict:
        names = ["n", "phi", "ux", "uy", "phi_tilde", "dphix", "dphiy", "lap", "mu", "Fx", "Fy"]
        arrs = {k: np.zeros((self.ny, self.nx)) for k in names}
        lib().o_fields(self.h, *[_ptr(arrs[k]) for k in names])
        return arrs

    def moments(self) -> dict:
        f = self.fields()
        return {k: f[k] for k in ("n", "phi", "ux", "uy")}

    def get_state(self):
        f = np.zeros((9, self.ny, self.nx))
        g = np.zeros((5, self.ny, self.nx))
        lib().o_get_state(self.h, _ptr(f), _ptr(g))
        return f, g

    def set_state(self, f, g, t: int = 0):
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        lib().o_set_state(self.h, _ptr(f), _ptr(g), int(t))

    def diag(self, row0: int):
        rec = np.zeros(6)
        cnt = np.zeros(self.ny, dtype=np.int64)
        uy = np.zeros(self.ny)
        lib().o_diag(self.h, int(row0), rec.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                     _ptr(cnt), _ptr(uy))
        return {"mass_n": rec[0], "mass_phi": rec[1], "mom_x": rec[2], "mom_y": rec[3],
                "max_u": rec[4], "nan_count": int(rec[5]), "row_count": cnt, "row_uy": uy}


# --------------------------------------------------------------------------
# Droplet diagnostics from the per-row ink profile.  The paper reports the
# breakup time and drop velocity (Results, Figs. 4-7) without defining how they
# are measured; this follows the row-segment reading stated in the design notes.
# --------------------------------------------------------------------------

def band_rows(width: float) -> int:
    """Rows of the head and of the tail of a drop: one interface width."""
    return max(1, int(math.ceil(width - 1e-9)))


def segments(row_count: np.ndarray, row_uy: np.ndarray, row0: int, a_min: float, band: int = 1) -> dict:
    """Split the rows y >= row0 into maximal runs with ink.  The run that
    contains row0 (the nozzle exit row) is attached; every other run with at
    least a_min ink nodes is a detached drop.  Returns the number of detached
    drops and, for the largest one, its ink count, summed u_y, highest and
    lowest rows, and the mean u_y of the ink in its top `band` rows (head)
    and in its bottom `band` rows (tail) -- the head and tail velocities of
    Fig. 3."""
    runs = []
    y = row0
    ny = len(row_count)
    while y < ny:
        if row_count[y] > 0:
            y1 = y
            while y1 < ny and row_count[y1] > 0:
                y1 += 1
            runs.append((y, y1))
            y = y1
        else:
            y += 1
    detached = []
    for (a, b) in runs:
        if a == row0:
            continue
        c = int(np.sum(row_count[a:b]))
        if c >= a_min:
            detached.append((c, float(np.sum(row_uy[a:b])), a, b))
    out = {"n_detached": len(detached), "largest_count": 0, "largest_uy": 0.0,
           "largest_top": -1, "largest_bottom": -1, "head_uy": 0.0, "tail_uy": 0.0}
    if detached:
        best = max(detached, key=lambda r: (r[0], -r[2]))
        a, b = best[2], best[3]
        h0, t1 = max(a, b - band), min(b, a + band)
        out.update(largest_count=best[0], largest_uy=best[1], largest_top=b - 1, largest_bottom=a,
                   head_uy=float(np.sum(row_uy[h0:b]) / np.sum(row_count[h0:b])),
                   tail_uy=float(np.sum(row_uy[a:t1]) / np.sum(row_count[a:t1])))
    return out


def breakup_summary(samples: list, ny: int, width: float, t_window=(1000, 3000),
                    t_volume=2000) -> dict:
    """Breakup step, drop velocity, drop volume and satellite flag from a time
    series of segment records (each a dict with 'step' plus the keys of
    :func:`segments`).  t_b is the first sample with a detached drop;
    v_drop averages the largest drop's mean u_y over samples in
    [t_b + 1000, t_b + 3000] (stopping once the drop top comes within 2W of
    the last row); V_drop is its ink count and the satellite flag is set when
    two or more drops are detached at the first sample at or after
    t_b + 2000.  drop_len is the rows spanned by the largest drop at t_b:
    the drop with its filament at breakup (Fig. 4)."""
    tb = -1
    for s in samples:
        if s["n_detached"] > 0:
            tb = s["step"]
            break
    out = {"breakup_step": tb, "v_drop": float("nan"), "vol_drop": 0, "satellite": 0, "drop_len": 0}
    if tb < 0:
        return out
    first = next(s for s in samples if s["step"] == tb)
    out["drop_len"] = int(first["largest_top"] - first["largest_bottom"] + 1)
    vs = []
    for s in samples:
        if tb + t_window[0] <= s["step"] <= tb + t_window[1] and s["largest_count"] > 0:
            if s["largest_top"] >= ny - 1 - 2 * width:
                break
            vs.append(s["largest_uy"] / s["largest_count"])
    if vs:
        out["v_drop"] = float(np.mean(vs))
    for s in samples:
        if s["step"] >= tb + t_volume:
            out["vol_drop"] = int(s["largest_count"])
            out["satellite"] = int(s["n_detached"] >= 2)
            break
    return out
