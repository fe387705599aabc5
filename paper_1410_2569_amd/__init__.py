"""MI355X-native (gfx950, FP64) wetting pseudopotential lattice Boltzmann step.

The hot path lives in liblbm.so (HIP kernels behind the C ABI of include/lbm.h); this package is
its thin Python binding.
"""
from .lbm import (ABI_VERSION, EOS, SCHEDULE, WALL, Batch, LBMError, Obs, Params, Sim,  # noqa: F401
                  Tune, autotune, cs_temperature, lib, make_params, maxwell_cs, workspace_size)

__all__ = ["Sim", "Batch", "Tune", "autotune", "Params", "Obs", "LBMError", "make_params", "maxwell_cs", "cs_temperature",
           "workspace_size", "lib", "WALL", "EOS", "SCHEDULE", "ABI_VERSION"]
