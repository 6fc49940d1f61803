"""MI355X (gfx950) entropic lattice Boltzmann hot path: KBC stream-and-collide sweep with
moving-wall Grad boundaries behind the C ABI in include/elbm.h.

The compute path is the HIP library ``libelbm.so`` built from ``csrc/``; ``elbm`` is its ctypes
binding.  Importing this package does not touch the GPU.
"""
from . import elbm  # noqa: F401
from .elbm import Lattice, ElbmError  # noqa: F401

__all__ = ["elbm", "Lattice", "ElbmError"]
