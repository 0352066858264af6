"""Python binding of the C ABI in ``include/inkjet_lbm.h`` (ctypes).

Argument marshalling only: every step of the update runs in the HIP library
``libinkjet_lbm.so``.  PyTorch provides device memory and streams; tensors
are passed to the library as raw device pointers on torch's current stream.
The module raises when the library is missing - there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libinkjet_lbm.so")

IJ_OK, IJ_ERR_INVALID_ARG, IJ_ERR_OOM, IJ_ERR_DEVICE, IJ_ERR_UNSTABLE, IJ_ERR_STATE = 0, -1, -2, -3, -4, -5
BC_PERIODIC, BC_OPEN = 0, 1

_INT_FIELDS = ["nx", "ny", "bc_y", "force_rows", "t_pos", "t_neg", "t_idle", "periodic_pulse",
               "nozzle_x0", "nozzle_w", "nozzle_len", "diag_row0", "diag_every"]
_DBL_FIELDS = ["rho_ink", "rho_amb", "sigma", "width", "gamma", "tau_ink", "tau_amb", "tau_phi",
               "theta_inner", "theta_outer", "f_pos", "f_neg", "u_limit"]


class IJParams(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in _INT_FIELDS] + [(k, ctypes.c_double) for k in _DBL_FIELDS]


class IJSample(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("mass_n", ctypes.c_double), ("mass_phi", ctypes.c_double),
                ("mom_x", ctypes.c_double), ("mom_y", ctypes.c_double), ("max_u", ctypes.c_double),
                ("nan_count", ctypes.c_int64), ("n_detached", ctypes.c_int64),
                ("largest_count", ctypes.c_int64), ("largest_uy", ctypes.c_double),
                ("largest_top", ctypes.c_int64), ("largest_bottom", ctypes.c_int64),
                ("head_uy", ctypes.c_double), ("tail_uy", ctypes.c_double)]


class IJDiag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("n_samples", ctypes.c_int64), ("breakup_step", ctypes.c_int64),
                ("v_drop", ctypes.c_double), ("vol_drop", ctypes.c_int64), ("satellite", ctypes.c_int64),
                ("unstable_step", ctypes.c_int64), ("last", IJSample), ("drop_len", ctypes.c_int64)]


class LBMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"inkjet_lbm error {code}: {msg}")
        self.code = code


_lib = None

# every symbol the header declares (checked by the CPU test-suite)
EXPORTS = ["ij_params_default", "ij_create", "ij_destroy", "ij_last_error", "ij_required_bytes",
           "ij_attach_buffers", "ij_set_wall", "ij_set_solid_mask", "ij_init_distance", "ij_init_phi", "ij_init_default",
           "ij_step", "ij_step_reference", "ij_time", "ij_get_moments", "ij_get_state", "ij_set_state",
           "ij_state_bytes", "ij_save_state", "ij_load_state",
           "ij_diag_sample", "ij_get_row_profile", "ij_get_samples", "ij_get_diagnostics", "ij_check",
           "ij_derived", "ij_set_tiling", "ij_autotune",
           "ij_batch_create", "ij_batch_destroy", "ij_batch_last_error", "ij_batch_size", "ij_batch_case",
           "ij_batch_time", "ij_batch_step", "ij_batch_set_graph", "ij_batch_set_tiling", "ij_batch_get_tiling",
           "ij_batch_autotune",
           "ij_mlp_create", "ij_mlp_create_seeded", "ij_mlp_destroy", "ij_mlp_last_error", "ij_mlp_param_count", "ij_mlp_set_weights",
           "ij_mlp_get_weights", "ij_mlp_set_scaling", "ij_mlp_gradients", "ij_mlp_train", "ij_mlp_predict",
           "ij_mlp_predict_noalloc",
           "ij3_create", "ij3_destroy", "ij3_last_error", "ij3_init", "ij3_step", "ij3_time", "ij3_get_moments",
           "ij3_get_state", "ij3_set_state", "ij3_state_bytes", "ij3_save_state", "ij3_load_state",
           "ij3_sample"]

_INT3 = ["nx", "ny", "nz", "bc_y", "force_rows", "t_pos", "t_neg", "t_idle", "periodic_pulse"]
_DBL3 = ["rho_ink", "rho_amb", "sigma", "width", "gamma", "tau_ink", "tau_amb", "tau_phi", "theta_inner",
         "theta_outer", "f_pos", "f_neg"]


class IJ3Params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in _INT3] + [(k, ctypes.c_double) for k in _DBL3]


class IJ3Drops(ctypes.Structure):
    _fields_ = [("n_detached", ctypes.c_int64), ("largest_count", ctypes.c_int64), ("largest_uy", ctypes.c_double),
                ("largest_top", ctypes.c_int64), ("largest_bottom", ctypes.c_int64), ("head_uy", ctypes.c_double),
                ("tail_uy", ctypes.c_double)]


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with `python -m paper_1702_04487_amd.build`")
    # torch first: its HIP runtime must be the one the library binds to (a
    # library loaded before torch pulls in the system runtime, and torch's
    # own then finds no GPU)
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    vp, i64, i32, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    sig = {
        "ij_params_default": (st, [ctypes.POINTER(IJParams)]),
        "ij_create": (st, [ctypes.POINTER(IJParams), ctypes.POINTER(vp)]),
        "ij_destroy": (None, [vp]),
        "ij_last_error": (ctypes.c_char_p, [vp]),
        "ij_required_bytes": (st, [ctypes.POINTER(IJParams), ctypes.POINTER(ctypes.c_size_t)]),
        "ij_attach_buffers": (st, [vp, vp, vp, ctypes.c_size_t]),
        "ij_set_wall": (st, [vp, vp]),
        "ij_set_solid_mask": (st, [vp, vp, i32]),
        "ij_init_distance": (st, [vp, vp, vp]),
        "ij_init_phi": (st, [vp, vp, vp, vp, vp]),
        "ij_init_default": (st, [vp, vp]),
        "ij_step": (st, [vp, i64, vp]),
        "ij_step_reference": (st, [vp, i64, vp]),
        "ij_time": (i64, [vp]),
        "ij_get_moments": (st, [vp, vp, vp, vp, vp, vp]),
        "ij_get_state": (st, [vp, vp, vp, vp]),
        "ij_set_state": (st, [vp, vp, vp, i64, vp]),
        "ij_state_bytes": (st, [vp, ctypes.POINTER(ctypes.c_size_t)]),
        "ij_save_state": (st, [vp, vp, ctypes.c_size_t, vp]),
        "ij_load_state": (st, [vp, vp, ctypes.c_size_t, vp]),
        "ij_diag_sample": (st, [vp, vp]),
        "ij_get_row_profile": (st, [vp, vp, vp, vp]),
        "ij_get_samples": (st, [vp, ctypes.POINTER(IJSample), i64, ctypes.POINTER(i64), vp]),
        "ij_get_diagnostics": (st, [vp, ctypes.POINTER(IJDiag), vp]),
        "ij_check": (st, [vp, vp]),
        "ij_derived": (st, [vp, ctypes.POINTER(ctypes.c_double)]),
        "ij_set_tiling": (st, [vp, i32, i32]),
        "ij_autotune": (st, [vp, i32, vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]),
        "ij_batch_create": (st, [ctypes.POINTER(IJParams), i32, ctypes.POINTER(vp)]),
        "ij_batch_destroy": (None, [vp]),
        "ij_batch_last_error": (ctypes.c_char_p, [vp]),
        "ij_batch_size": (i32, [vp]),
        "ij_batch_case": (st, [vp, i32, ctypes.POINTER(vp)]),
        "ij_batch_time": (i64, [vp]),
        "ij_batch_step": (st, [vp, i64, vp]),
        "ij_batch_set_graph": (st, [vp, i32]),
        "ij_batch_set_tiling": (st, [vp, i32, i32, i32, i32]),
        "ij_batch_get_tiling": (st, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                     ctypes.POINTER(i32)]),
        "ij_batch_autotune": (st, [vp, i32, vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                   ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]),
        "ij_mlp_create": (st, [i32, ctypes.POINTER(vp)]),
        "ij_mlp_create_seeded": (st, [i32, ctypes.c_uint64, ctypes.POINTER(vp)]),
        "ij_mlp_destroy": (None, [vp]),
        "ij_mlp_last_error": (ctypes.c_char_p, [vp]),
        "ij_mlp_param_count": (i32, []),
        "ij_mlp_set_weights": (st, [vp, i32, vp]),
        "ij_mlp_get_weights": (st, [vp, i32, vp]),
        "ij_mlp_set_scaling": (st, [vp, vp, vp, vp, vp]),
        "ij_mlp_gradients": (st, [vp, vp, vp, i32, vp, vp, vp]),
        "ij_mlp_train": (st, [vp, vp, vp, i32, vp, i32, i32, ctypes.c_float, vp, vp]),
        "ij_mlp_predict": (st, [vp, vp, i64, vp, vp, vp, vp]),
        "ij_mlp_predict_noalloc": (st, [vp, vp, i64, vp, vp, vp]),
        "ij3_create": (st, [ctypes.POINTER(IJ3Params), vp, ctypes.POINTER(vp)]),
        "ij3_destroy": (None, [vp]),
        "ij3_last_error": (ctypes.c_char_p, [vp]),
        "ij3_init": (st, [vp, vp, i32, vp, vp, vp, vp]),
        "ij3_step": (st, [vp, i64, vp]),
        "ij3_time": (i64, [vp]),
        "ij3_get_moments": (st, [vp, vp, vp, vp, vp, vp, vp]),
        "ij3_get_state": (st, [vp, vp, vp, vp]),
        "ij3_set_state": (st, [vp, vp, vp, i64, vp]),
        "ij3_state_bytes": (st, [vp, ctypes.POINTER(ctypes.c_size_t)]),
        "ij3_save_state": (st, [vp, vp, ctypes.c_size_t, vp]),
        "ij3_load_state": (st, [vp, vp, ctypes.c_size_t, vp]),
        "ij3_sample": (st, [vp, i64, vp, vp, vp, i64, i64, ctypes.POINTER(IJ3Drops), vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def to_params(d: dict) -> IJParams:
    p = IJParams()
    load().ij_params_default(ctypes.byref(p))
    # a dict without nozzle fields describes an all-fluid lattice (walls come from set_wall)
    p.nozzle_w = 0
    p.nozzle_x0 = 0
    p.nozzle_len = 0
    p.diag_row0 = 0
    for k in _INT_FIELDS + _DBL_FIELDS:
        if k in d:
            setattr(p, k, d[k])
    return p


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t) -> Optional[ctypes.c_void_p]:
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous() and t.dtype.is_floating_point
    return ctypes.c_void_p(t.data_ptr())


class Sim:
    """One lattice on the GPU, owned by the library (or by caller tensors
    passed to :meth:`attach`)."""

    def __init__(self, params: dict, wall: Optional[np.ndarray] = None, _handle=None):
        import torch
        self.L = load()
        self.params = dict(params)
        self.nx, self.ny = int(params["nx"]), int(params["ny"])
        self._p = to_params(params)
        self._owned = _handle is None
        if _handle is None:
            h = ctypes.c_void_p()
            r = self.L.ij_create(ctypes.byref(self._p), ctypes.byref(h))
            if r != IJ_OK:
                raise LBMError(r, self.L.ij_last_error(None).decode())
        else:
            h = _handle
        self.h = h
        self._keep = []
        self.device = torch.device("cuda", torch.cuda.current_device())
        if wall is not None:
            self.set_wall(wall)

    def _check(self, r: int):
        if r != IJ_OK:
            raise LBMError(r, self.L.ij_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            if self._owned:
                self.L.ij_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ set-up
    def set_wall(self, wall):
        """Wall mask [ny, nx] of IJ_FLUID / IJ_WALL_INNER / IJ_WALL_OUTER: a
        host array (:c:func:`ij_set_wall`) or a uint8 tensor on the device
        (:c:func:`ij_set_solid_mask` with on_device = 1)."""
        if hasattr(wall, "is_cuda") and wall.is_cuda:
            import torch
            assert wall.dtype == torch.uint8 and tuple(wall.shape) == (self.ny, self.nx)
            w = wall.contiguous()
            self._check(self.L.ij_set_solid_mask(self.h, ctypes.c_void_p(w.data_ptr()), 1))
            return
        w = np.ascontiguousarray(wall, dtype=np.uint8)
        assert w.shape == (self.ny, self.nx)
        self._check(self.L.ij_set_wall(self.h, w.ctypes.data_as(ctypes.c_void_p)))

    def set_tiling(self, waves_x: int = 0, rows_per_block: int = 0):
        self._check(self.L.ij_set_tiling(self.h, int(waves_x), int(rows_per_block)))

    def autotune(self, trial_steps: int = 20, stream=None):
        """Returns (waves_x, rows_per_block, ms per step)."""
        w, r, ms = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_double(0)
        self._check(self.L.ij_autotune(self.h, int(trial_steps), _stream_ptr(stream), ctypes.byref(w),
                                       ctypes.byref(r), ctypes.byref(ms)))
        return int(w.value), int(r.value), float(ms.value)

    def attach(self, a, b):
        """Use two caller tensors (torch, uint8/float, contiguous, on the
        device) as the distribution buffers."""
        need = self.required_bytes()
        for t in (a, b):
            assert t.is_cuda and t.is_contiguous() and t.numel() * t.element_size() >= need
        self._keep = [a, b]
        self._check(self.L.ij_attach_buffers(self.h, ctypes.c_void_p(a.data_ptr()),
                                             ctypes.c_void_p(b.data_ptr()), need))

    def required_bytes(self) -> int:
        n = ctypes.c_size_t(0)
        r = self.L.ij_required_bytes(ctypes.byref(self._p), ctypes.byref(n))
        if r != IJ_OK:
            raise LBMError(r, self.L.ij_last_error(None).decode())
        return int(n.value)

    def derived(self) -> dict:
        out = (ctypes.c_double * 8)()
        self._check(self.L.ij_derived(self.h, out))
        keys = ["phi_star", "n0", "beta", "kappa", "q", "wet_inner", "wet_outer", "mobility"]
        return dict(zip(keys, list(out)))

    def _dev(self, a, shape=None):
        """float32 contiguous device copy, checked against the shape the
        kernels will index ([ny][nx] unless given)."""
        import torch
        if isinstance(a, torch.Tensor):
            t = a.to(device=self.device, dtype=torch.float32).contiguous()
        else:
            t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=self.device)
        want = tuple(shape) if shape is not None else (self.ny, self.nx)
        if tuple(t.shape) != want:
            raise ValueError(f"array of shape {tuple(t.shape)} where {want} is required")
        return t

    def init_distance(self, d, stream=None):
        dd = self._dev(d)
        self._check(self.L.ij_init_distance(self.h, _dptr(dd), _stream_ptr(stream)))
        self._keep_init = dd

    def init_phi(self, phi, ux=None, uy=None, stream=None):
        p, x, y = self._dev(phi), None if ux is None else self._dev(ux), None if uy is None else self._dev(uy)
        self._check(self.L.ij_init_phi(self.h, _dptr(p), _dptr(x), _dptr(y), _stream_ptr(stream)))
        self._keep_init = (p, x, y)

    def init_default(self, stream=None):
        self._check(self.L.ij_init_default(self.h, _stream_ptr(stream)))

    # ------------------------------------------------------------ stepping
    def step(self, n: int = 1, stream=None):
        self._check(self.L.ij_step(self.h, int(n), _stream_ptr(stream)))

    def step_reference(self, n: int = 1, stream=None):
        self._check(self.L.ij_step_reference(self.h, int(n), _stream_ptr(stream)))

    @property
    def t(self) -> int:
        return int(self.L.ij_time(self.h))

    # ------------------------------------------------------------ readback
    def moments(self, stream=None) -> dict:
        import torch
        out = {k: torch.empty((self.ny, self.nx), device=self.device, dtype=torch.float32)
               for k in ("n", "phi", "ux", "uy")}
        self._check(self.L.ij_get_moments(self.h, _dptr(out["n"]), _dptr(out["phi"]), _dptr(out["ux"]),
                                          _dptr(out["uy"]), _stream_ptr(stream)))
        return out

    def state(self, stream=None):
        import torch
        f = torch.empty((9, self.ny, self.nx), device=self.device, dtype=torch.float32)
        g = torch.empty((5, self.ny, self.nx), device=self.device, dtype=torch.float32)
        self._check(self.L.ij_get_state(self.h, _dptr(f), _dptr(g), _stream_ptr(stream)))
        return f, g

    def set_state(self, f, g, t: int = 0, stream=None):
        ff, gg = self._dev(f, (9, self.ny, self.nx)), self._dev(g, (5, self.ny, self.nx))
        self._check(self.L.ij_set_state(self.h, _dptr(ff), _dptr(gg), int(t), _stream_ptr(stream)))
        self._keep_state = (ff, gg)

    def save_state(self, stream=None) -> bytes:
        """Checkpoint blob of the current state (:c:func:`ij_save_state`)."""
        n = ctypes.c_size_t(0)
        self._check(self.L.ij_state_bytes(self.h, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(self.L.ij_save_state(self.h, buf, n.value, _stream_ptr(stream)))
        return buf.raw

    def load_state(self, blob: bytes, stream=None):
        """Resume from a blob of :meth:`save_state` (:c:func:`ij_load_state`)."""
        self._check(self.L.ij_load_state(self.h, ctypes.c_char_p(blob), len(blob), _stream_ptr(stream)))

    def diag_sample(self, stream=None):
        self._check(self.L.ij_diag_sample(self.h, _stream_ptr(stream)))

    def row_profile(self, stream=None):
        cnt = np.zeros(self.ny, dtype=np.int64)
        uy = np.zeros(self.ny, dtype=np.float64)
        self._check(self.L.ij_get_row_profile(self.h, cnt.ctypes.data_as(ctypes.c_void_p),
                                              uy.ctypes.data_as(ctypes.c_void_p), _stream_ptr(stream)))
        return cnt, uy

    def samples(self, stream=None) -> list:
        n = ctypes.c_int64(0)
        self._check(self.L.ij_get_samples(self.h, None, 0, ctypes.byref(n), _stream_ptr(stream)))
        arr = (IJSample * max(1, n.value))()
        self._check(self.L.ij_get_samples(self.h, arr, n.value, ctypes.byref(n), _stream_ptr(stream)))
        return [{k: getattr(arr[i], k) for k, _ in IJSample._fields_} for i in range(n.value)]

    def diagnostics(self, stream=None) -> dict:
        d = IJDiag()
        self._check(self.L.ij_get_diagnostics(self.h, ctypes.byref(d), _stream_ptr(stream)))
        out = {k: getattr(d, k) for k, _ in IJDiag._fields_ if k != "last"}
        out["last"] = {k: getattr(d.last, k) for k, _ in IJSample._fields_}
        return out

    def check(self, stream=None) -> int:
        return int(self.L.ij_check(self.h, _stream_ptr(stream)))


class Batch:
    """Independent lattices stepped together (:c:func:`ij_batch_create`).
    ``cases`` is a list of parameter dicts; ``walls`` an optional list of
    wall masks (None entries keep the nozzle of the parameters)."""

    def __init__(self, cases: list, walls: Optional[list] = None):
        self.L = load()
        n = len(cases)
        arr = (IJParams * n)()
        for i, c in enumerate(cases):
            arr[i] = to_params(c)
        h = ctypes.c_void_p()
        r = self.L.ij_batch_create(arr, n, ctypes.byref(h))
        if r != IJ_OK:
            raise LBMError(r, self.L.ij_batch_last_error(None).decode())
        self.h = h
        self.cases = []
        for i, c in enumerate(cases):
            ch = ctypes.c_void_p()
            self._check(self.L.ij_batch_case(self.h, i, ctypes.byref(ch)))
            w = None if walls is None else walls[i]
            self.cases.append(Sim(c, w, _handle=ch))

    def _check(self, r: int):
        if r != IJ_OK:
            raise LBMError(r, self.L.ij_batch_last_error(self.h).decode())

    def __len__(self):
        return len(self.cases)

    def close(self):
        if getattr(self, "h", None):
            for c in self.cases:
                c.h = None
            self.L.ij_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def t(self) -> int:
        return int(self.L.ij_batch_time(self.h))

    def step(self, n: int = 1, stream=None):
        self._check(self.L.ij_batch_step(self.h, int(n), _stream_ptr(stream)))

    def set_graph(self, steps_per_graph: int):
        self._check(self.L.ij_batch_set_graph(self.h, int(steps_per_graph)))

    def set_tiling(self, waves_x: int, rows_per_block: int, mixed_strips: bool = False, persistent: bool = True):
        self._check(self.L.ij_batch_set_tiling(self.h, int(waves_x), int(rows_per_block), int(bool(mixed_strips)),
                                               int(bool(persistent))))

    def tiling(self):
        """(waves_x, rows_per_block, mixed_strips, persistent)."""
        w, r, m, p = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        self._check(self.L.ij_batch_get_tiling(self.h, ctypes.byref(w), ctypes.byref(r), ctypes.byref(m),
                                               ctypes.byref(p)))
        return int(w.value), int(r.value), bool(m.value), bool(p.value)

    def autotune(self, trial_steps: int = 20, stream=None):
        """Returns (waves_x, rows_per_block, mixed_strips, persistent, ms per
        step or -1 if cached)."""
        w, r, m, p, ms = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_double(0)
        self._check(self.L.ij_batch_autotune(self.h, int(trial_steps), _stream_ptr(stream), ctypes.byref(w),
                                             ctypes.byref(r), ctypes.byref(m), ctypes.byref(p), ctypes.byref(ms)))
        return int(w.value), int(r.value), bool(m.value), bool(p.value), float(ms.value)


MLP_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")
MLP_SHAPES = {"W1": (128, 7), "b1": (128,), "W2": (128, 128), "b2": (128,), "W3": (4, 128), "b3": (4,)}


def pack_params(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], np.float64).reshape(-1) for k in MLP_NAMES])


def unpack_params(v: np.ndarray) -> dict:
    out, off = {}, 0
    for k in MLP_NAMES:
        n = int(np.prod(MLP_SHAPES[k]))
        out[k] = v[off:off + n].reshape(MLP_SHAPES[k]).copy()
        off += n
    return out


class MLP:
    """Ensemble of surrogate networks (:c:func:`ij_mlp_create`)."""

    def __init__(self, n_members: int = 4, seed: Optional[int] = None):
        """Zero parameters, or with `seed` the seeded initial parameters of
        :c:func:`ij_mlp_create_seeded`."""
        import torch
        self.L = load()
        h = ctypes.c_void_p()
        if seed is None:
            r = self.L.ij_mlp_create(int(n_members), ctypes.byref(h))
        else:
            r = self.L.ij_mlp_create_seeded(int(n_members), ctypes.c_uint64(int(seed) & (2 ** 64 - 1)), ctypes.byref(h))
        if r != IJ_OK:
            raise LBMError(r, self.L.ij_mlp_last_error(None).decode())
        self.h = h
        self.n_members = int(n_members)
        self.n_params = int(self.L.ij_mlp_param_count())
        self.device = torch.device("cuda", torch.cuda.current_device())

    def _check(self, r: int):
        if r != IJ_OK:
            raise LBMError(r, self.L.ij_mlp_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.L.ij_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _f32(self, a, cols):
        import torch
        t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=self.device) \
            if not isinstance(a, torch.Tensor) else a.to(self.device, torch.float32).contiguous()
        if t.dim() != 2 or t.shape[1] != cols:
            raise ValueError(f"expected an [n, {cols}] array, got {tuple(t.shape)}")
        return t

    def set_weights(self, member: int, params: dict):
        v = np.ascontiguousarray(pack_params(params))
        assert v.size == self.n_params
        self._check(self.L.ij_mlp_set_weights(self.h, int(member), v.ctypes.data_as(ctypes.c_void_p)))

    def get_weights(self, member: int) -> dict:
        v = np.zeros(self.n_params)
        self._check(self.L.ij_mlp_get_weights(self.h, int(member), v.ctypes.data_as(ctypes.c_void_p)))
        return unpack_params(v)

    def set_scaling(self, x_mean, x_std, y_mean, y_std):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x_mean, x_std, y_mean, y_std)]
        assert [a.size for a in arrs] == [7, 7, 3, 3]
        self._keep_scaling = arrs
        self._check(self.L.ij_mlp_set_scaling(self.h, *[a.ctypes.data_as(ctypes.c_void_p) for a in arrs]))

    def gradients(self, x, y, stream=None):
        """(loss [members], list of packed-gradient dicts per member)."""
        xt, yt = self._f32(x, 7), self._f32(y, 4)
        g = np.zeros((self.n_members, self.n_params))
        l = np.zeros(self.n_members)
        self._check(self.L.ij_mlp_gradients(self.h, _dptr(xt), _dptr(yt), int(xt.shape[0]),
                                            g.ctypes.data_as(ctypes.c_void_p), l.ctypes.data_as(ctypes.c_void_p),
                                            _stream_ptr(stream)))
        return l, [unpack_params(g[k]) for k in range(self.n_members)]

    def train(self, x, y, idx, lr: float, stream=None):
        """idx: int array [n_members, steps, batch]; returns the per-step
        losses [n_members, steps] (a device tensor)."""
        import torch
        xt, yt = self._f32(x, 7), self._f32(y, 4)
        it = torch.as_tensor(np.ascontiguousarray(idx, dtype=np.int32), device=self.device)
        if it.dim() != 3 or it.shape[0] != self.n_members:
            raise ValueError("idx must be [n_members, steps, batch]")
        loss = torch.zeros((self.n_members, it.shape[1]), device=self.device, dtype=torch.float32)
        self._check(self.L.ij_mlp_train(self.h, _dptr(xt), _dptr(yt), int(xt.shape[0]),
                                        ctypes.c_void_p(it.data_ptr()), int(it.shape[1]), int(it.shape[2]),
                                        float(lr), _dptr(loss), _stream_ptr(stream)))
        self._keep_train = (xt, yt, it)
        return loss

    def predict(self, x, members: bool = False, stream=None):
        """(mean [n, 4], spread [n, 4]) device tensors, and the per-member
        outputs [n_members, n, 4] when members is set."""
        import torch
        xt = self._f32(x, 7)
        n = int(xt.shape[0])
        mean = torch.empty((n, 4), device=self.device, dtype=torch.float32)
        spread = torch.empty((n, 4), device=self.device, dtype=torch.float32)
        mem = torch.empty((self.n_members, n, 4), device=self.device, dtype=torch.float32) if members else None
        self._check(self.L.ij_mlp_predict(self.h, _dptr(xt), n, _dptr(mean), _dptr(spread),
                                          _dptr(mem) if mem is not None else None, _stream_ptr(stream)))
        self._keep_pred = xt
        return (mean, spread, mem) if members else (mean, spread)

    def predict_into(self, x, mean, spread, stream=None):
        """Prediction into caller tensors (mean, spread: [n, 4] float32 on the
        device) through :c:func:`ij_mlp_predict_noalloc`, which allocates
        nothing; x must already be a contiguous float32 [n, 7] device tensor."""
        import torch
        n = int(x.shape[0])
        for t in (x, mean, spread):
            assert isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous() and t.dtype == torch.float32
        assert tuple(x.shape) == (n, 7) and tuple(mean.shape) == (n, 4) and tuple(spread.shape) == (n, 4)
        self._check(self.L.ij_mlp_predict_noalloc(self.h, _dptr(x), n, _dptr(mean), _dptr(spread),
                                                  _stream_ptr(stream)))
