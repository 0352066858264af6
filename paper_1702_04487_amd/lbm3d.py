"""Python binding of the three-dimensional entry points (``ij3_*`` in
``include/inkjet_lbm.h``): D3Q19 / D3Q7 lattices for round nozzles.

Argument marshalling only: every step runs in the HIP library.  Arrays are
indexed ``[y, z, x]`` (x fastest); tensors go to the library as raw device
pointers on torch's current stream.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional

import numpy as np

from .lbm import IJ_OK, IJ3Drops, IJ3Params, LBMError, _INT3, _DBL3, _dptr, _stream_ptr, load

Q, QG = 19, 7


def to_params3(d: dict) -> IJ3Params:
    p = IJ3Params()
    for k in _INT3 + _DBL3:
        setattr(p, k, d[k])
    return p


class Sim3D:
    """One three-dimensional lattice on the GPU, owned by the library."""

    def __init__(self, params: dict, wall: Optional[np.ndarray] = None):
        import torch
        self.L = load()
        self.params = dict(params)
        self.nx, self.ny, self.nz = int(params["nx"]), int(params["ny"]), int(params["nz"])
        self.shape = (self.ny, self.nz, self.nx)
        self._p = to_params3(params)
        w = None
        if wall is not None:
            w = np.ascontiguousarray(wall, dtype=np.uint8)
            if w.shape != self.shape:
                raise ValueError(f"wall of shape {w.shape} where {self.shape} is required")
        h = ctypes.c_void_p()
        r = self.L.ij3_create(ctypes.byref(self._p), None if w is None else w.ctypes.data_as(ctypes.c_void_p),
                              ctypes.byref(h))
        if r != IJ_OK:
            raise LBMError(r, self.L.ij3_last_error(None).decode())
        self.h = h
        self.device = torch.device("cuda", torch.cuda.current_device())

    def _check(self, r: int):
        if r != IJ_OK:
            raise LBMError(r, self.L.ij3_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.L.ij3_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, shape=None):
        import torch
        if isinstance(a, torch.Tensor):
            t = a.to(device=self.device, dtype=torch.float32).contiguous()
        else:
            t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=self.device)
        want = tuple(shape) if shape is not None else self.shape
        if tuple(t.shape) != want:
            raise ValueError(f"array of shape {tuple(t.shape)} where {want} is required")
        return t

    def _init(self, src, from_distance, ux, uy, uz, stream):
        s = self._dev(src)
        u = [None if a is None else self._dev(a) for a in (ux, uy, uz)]
        self._check(self.L.ij3_init(self.h, _dptr(s), int(from_distance), *(_dptr(a) for a in u),
                                    _stream_ptr(stream)))
        self._keep_init = (s, u)

    def init_distance(self, d, stream=None):
        self._init(d, 1, None, None, None, stream)

    def init_phi(self, phi, ux=None, uy=None, uz=None, stream=None):
        self._init(phi, 0, ux, uy, uz, stream)

    def step(self, n: int = 1, stream=None):
        self._check(self.L.ij3_step(self.h, int(n), _stream_ptr(stream)))

    @property
    def t(self) -> int:
        return int(self.L.ij3_time(self.h))

    def moments(self, stream=None) -> dict:
        import torch
        out = {k: torch.empty(self.shape, dtype=torch.float32, device=self.device)
               for k in ("n", "phi", "ux", "uy", "uz")}
        self._check(self.L.ij3_get_moments(self.h, *(_dptr(out[k]) for k in ("n", "phi", "ux", "uy", "uz")),
                                           _stream_ptr(stream)))
        return out

    def state(self, stream=None):
        import torch
        f = torch.empty((Q,) + self.shape, dtype=torch.float32, device=self.device)
        g = torch.empty((QG,) + self.shape, dtype=torch.float32, device=self.device)
        self._check(self.L.ij3_get_state(self.h, _dptr(f), _dptr(g), _stream_ptr(stream)))
        return f, g

    def set_state(self, f, g, t: int = 0, stream=None):
        ft, gt = self._dev(f, (Q,) + self.shape), self._dev(g, (QG,) + self.shape)
        self._check(self.L.ij3_set_state(self.h, _dptr(ft), _dptr(gt), int(t), _stream_ptr(stream)))
        self._keep_state = (ft, gt)

    def save_state(self, stream=None) -> bytes:
        """Checkpoint blob of the current state (:c:func:`ij3_save_state`)."""
        n = ctypes.c_size_t(0)
        self._check(self.L.ij3_state_bytes(self.h, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(self.L.ij3_save_state(self.h, buf, n.value, _stream_ptr(stream)))
        return buf.raw

    def load_state(self, blob: bytes, stream=None):
        """Resume from a blob of :meth:`save_state` (:c:func:`ij3_load_state`)."""
        self._check(self.L.ij3_load_state(self.h, ctypes.c_char_p(blob), len(blob), _stream_ptr(stream)))

    def sample(self, row0: int = 0, a_min: Optional[int] = None, band: Optional[int] = None, stream=None) -> dict:
        """Sums, per-row ink profile and droplet segments of the current
        state; a drop needs a_min ink nodes (default 4 W^3), head and tail
        velocities average over `band` rows (default ceil(W))."""
        w = float(self.params["width"])
        a_min = int(round(4 * w ** 3)) if a_min is None else int(a_min)
        band = int(math.ceil(w)) if band is None else int(band)
        rec = np.zeros(7)
        cnt = np.zeros(self.ny, dtype=np.int64)
        uy = np.zeros(self.ny)
        d = IJ3Drops()
        self._check(self.L.ij3_sample(self.h, int(row0), rec.ctypes.data_as(ctypes.c_void_p),
                                      cnt.ctypes.data_as(ctypes.c_void_p), uy.ctypes.data_as(ctypes.c_void_p),
                                      a_min, band, ctypes.byref(d), _stream_ptr(stream)))
        drops = {k: getattr(d, k) for k, _ in IJ3Drops._fields_}
        return dict(mass_n=rec[0], mass_phi=rec[1], mom=rec[2:5].copy(), max_u=rec[5], nan_count=int(rec[6]),
                    row_count=cnt, row_uy=uy, drops=drops)
