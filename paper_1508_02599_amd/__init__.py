"""MI355X-native classical and all-floating FETI (Augustin, Holzapfel, Steinbach).

The solver lives in ``libfeti.so`` (HIP kernels for gfx950 behind the C ABI of
``include/feti.h``); :mod:`paper_1508_02599_amd.feti` is its ctypes binding.
"""
from .feti import (Problem, FetiError, load_library, feti_setup, feti_factor, feti_solve,
                   feti_newton_step, feti_footprint, feti_destroy, LIB_PATH)

__all__ = ["Problem", "FetiError", "load_library", "feti_setup", "feti_factor", "feti_solve",
           "feti_newton_step", "feti_footprint", "feti_destroy", "LIB_PATH"]
