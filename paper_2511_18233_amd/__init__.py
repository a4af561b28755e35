"""MI355X (gfx950) TDDFT-ris gradient / derivative-coupling hot path.

The compute lives in libris_hip.so (HIP kernels behind the C ABI of
include/ris.h); ``paper_2511_18233_amd.ris`` is its ctypes binding.
"""
from .ris import EXPORTS, LIB_PATH, RisContext, RisError, load_library, solve_problem  # noqa: F401

__all__ = ["RisContext", "RisError", "load_library", "solve_problem", "EXPORTS", "LIB_PATH"]
