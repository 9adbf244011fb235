"""MI355X-native Jacobi3D hot path (arXiv 2102.12416, section 4.3, one GPU).

libjc.so (HIP kernels + host runtime, C-ABI in include/jc.h) does the work;
this package binds it with ctypes and supplies torch device memory and
streams.  Importing it fails if libjc.so has not been built.
"""
from . import _lib
from ._lib import JcError
from .solver import Group, Solver, footprint, min_surface_parts, synth_field

__all__ = ["Group", "Solver", "JcError", "footprint", "min_surface_parts", "synth_field", "_lib"]
