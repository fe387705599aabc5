"""MI355X-native (gfx950, FP64) wetting pseudopotential lattice Boltzmann step.

The hot path lives in liblbm.so (HIP kernels behind the C ABI of include/lbm.h); this package is
its thin Python binding.
"""
from .lbm import (ABI_VERSION, EOS, SCHEDULE, WALL, WALLS, Batch, Droplets, LBMError, Obs,  # noqa: F401
                  Params, Sim, Tune, autotune, cs_temperature, lib, make_droplets, make_params,
                  maxwell_cs,
                  observables_of_state, piecewise_spinodals, workspace_size)

__all__ = ["Sim", "Batch", "Tune", "autotune", "Params", "Obs", "LBMError", "make_params",
           "Droplets", "make_droplets",
           "maxwell_cs", "cs_temperature", "piecewise_spinodals", "workspace_size", "observables_of_state", "lib", "WALL",
           "WALLS", "EOS", "SCHEDULE", "ABI_VERSION"]
