"""MI355X (gfx950) binary-fluid lattice Boltzmann library for inkjet droplet
formation (He, Yang, Qin, Wen & Zhang, arXiv:1702.04487).

The update runs in HIP kernels behind the C ABI of ``include/inkjet_lbm.h``;
:mod:`paper_1702_04487_amd.lbm` is its Python binding.
"""
from . import lbm  # noqa: F401

__all__ = ["lbm"]
