"""lbm355: D3Q19 lattice Boltzmann propagation schemes as HIP kernels for MI355X (gfx950).

The compute path is liblbm355.so (C ABI in include/lbm355.h); this package is
its Python binding.  Importing it loads the library and fails loudly when it
is not built.
"""
from . import _lib
from ._lib import LbmError, load
from .grid import Grid, lattice, model_bytes, stream_copy
from .batch import Batch

__all__ = ["Batch", "Grid", "LbmError", "lattice", "load", "model_bytes", "stream_copy", "_lib"]

load()
