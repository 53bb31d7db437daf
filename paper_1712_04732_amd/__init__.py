"""MI355X-native Spectral Ewald k-space library (arXiv:1712.04732).

The computation runs in libse_mi355x.so (hand-written gfx950 HIP kernels behind
the C ABI of include/se.h).  This package holds the ctypes binding (_lib), the
torch-facing plans (k space, real space), the autograd adjoint and total
energy (api), and the build script (build_lib).
"""
from . import _lib
from .api import (EwaldEnergy, RealSpace, SEEnergy, SEPotential, SpectralEwald, SpectralEwaldBatch,
                  params_for_tolerance, params_recipe)

__all__ = ["EwaldEnergy", "RealSpace", "SpectralEwald", "SpectralEwaldBatch", "SEEnergy", "SEPotential",
           "params_for_tolerance", "params_recipe", "_lib"]
