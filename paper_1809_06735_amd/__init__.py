"""MI355X-native D2Q9 lattice-Boltzmann step and sub-volume balance diagnostic.

The computation lives in the HIP library ``libpaper_lbm.so`` (C ABI in
``include/lbm.h``); this package only marshals arguments to it.  Nothing here
falls back to the CPU: without the built library or without a GPU every entry
point raises.
"""
from ._lib import LBMError, LIB_PATH, TERM_NAMES, load  # noqa: F401
from .sim import (Simulation, Simulation3D, balance_fields, balance_fields_noalloc,  # noqa: F401
                  configuration_statistics, copy_bandwidth, energy_spectrum, sample_configurations,
                  stats_to_dict)

__all__ = ["Simulation", "Simulation3D", "balance_fields", "balance_fields_noalloc", "configuration_statistics", "copy_bandwidth",
           "energy_spectrum", "sample_configurations", "stats_to_dict", "LBMError", "load", "LIB_PATH",
           "TERM_NAMES"]
