"""MI355X-native THC-MPO H|psi> library (arXiv 2409.12708 hot path).

The compute lives in libthck.so (hand-written HIP for gfx950, C ABI in
include/thck.h); ``thck`` is the ctypes binding.
"""
from .thck import (Context, DeviceMPS, Krylov, ThcError, ThcStats, capacity, load_library,  # noqa: F401
                   make_opts, EXPORTS, FLAG_SVD_JACOBI, FLAG_TIME_KERNELS)

__all__ = ["Context", "DeviceMPS", "Krylov", "ThcError", "ThcStats", "capacity", "load_library", "make_opts",
           "EXPORTS", "FLAG_SVD_JACOBI", "FLAG_TIME_KERNELS"]
