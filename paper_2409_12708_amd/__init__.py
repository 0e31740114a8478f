"""MI355X-native THC-MPO H|psi> library (arXiv 2409.12708 hot path).

The compute lives in libthck.so (hand-written HIP for gfx950, C ABI in
include/thck.h); ``thck`` is the ctypes binding.
"""
from .thck import (Context, DeviceMPS, Krylov, ThcEnergy, ThcError, ThcStats, capacity,  # noqa: F401
                   evolve, load_library, make_opts, thc_energy, EXPORTS, FLAG_GRAPHS, FLAG_SVD_JACOBI, FLAG_SYTRD_ONE_STAGE,
                   FLAG_TIME_KERNELS, FLAG_TWO_STREAMS)

__all__ = ["Context", "DeviceMPS", "Krylov", "ThcEnergy", "ThcError", "ThcStats", "capacity", "evolve", "load_library",
           "make_opts", "thc_energy", "EXPORTS", "FLAG_GRAPHS", "FLAG_SVD_JACOBI", "FLAG_SYTRD_ONE_STAGE",
           "FLAG_TIME_KERNELS", "FLAG_TWO_STREAMS"]
