"""MI355X-native split-step propagator for two interacting electrons in a
quantum-Hall Hong-Ou-Mandel interferometer (arXiv 1903.02581).

The compute path is libhom4d.so (HIP, gfx950) behind the C ABI in
include/hom4d.h; this package is its thin Python binding.
"""
from .hom4d import (COULOMB_DIRECT, COULOMB_TABLE, FP64, MIXED, Hom4dError,  # noqa: F401
                    Propagator, load_library, make_cfg)

__all__ = ["Propagator", "Hom4dError", "load_library", "make_cfg", "BunchingLoss",
           "saddle_potential"]


def __getattr__(name):
    if name in ("BunchingLoss", "saddle_potential", "bunching_loss"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
