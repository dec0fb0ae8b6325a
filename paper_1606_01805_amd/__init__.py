"""MI355X (gfx950) implementation of the coupled lattice-Boltzmann / MLS
immersed-boundary particle-transport method of Coclite et al.

The hot path lives in the HIP library libpaper_lbm.so behind the C ABI of
include/lbm.h; this package is its Python binding.  There is no CPU fallback:
importing Solver loads the library and fails loudly if it has not been built.
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpaper_lbm.so")


def __getattr__(name):
    if name in ("Solver", "channel_config"):
        from . import solver
        return getattr(solver, name)
    if name in ("lib", "LBMError"):
        from . import _lib
        return getattr(_lib, name)
    raise AttributeError(name)
