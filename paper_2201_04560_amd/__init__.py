"""MI355X-native pseudopotential lattice-Boltzmann step for liquid-vapour
phase change (Jaramillo, Mapelli, Cabezas-Gomez): a HIP library for gfx950
behind the C-ABI of include/lbm_pp.h, with a thin ctypes binding.

Importing the package does not load the library; the first call does, and
raises ImportError if the library has not been built.
"""
from ._native import (LBM_FP32_SHIFTED, LBM_FP64, LBM_WALL_MODIFIED_PSI, LBM_WALL_PSI_BASED,
                      T_ADIABATIC, T_DIRICHLET, T_FREE, LbmError, LbmParams, lib)
from .sim import (Batch, Lattice, buffer_bytes, fit_sigma, make_params, planar_gamma,
                  pr_critical_temperature, pr_latent_heat, pr_maxwell, refinement_level, stefan_beta)

from .adjoint import HeaterAdjoint, HeaterProblem, evaporated_mass

__all__ = ["HeaterAdjoint", "HeaterProblem", "evaporated_mass", "Lattice", "Batch", "refinement_level", "LbmParams", "LbmError", "make_params", "buffer_bytes", "lib",
           "pr_critical_temperature", "pr_maxwell", "fit_sigma", "planar_gamma", "pr_latent_heat",
           "stefan_beta",
           "LBM_FP64", "LBM_FP32_SHIFTED", "LBM_WALL_PSI_BASED", "LBM_WALL_MODIFIED_PSI",
           "T_FREE", "T_DIRICHLET", "T_ADIABATIC"]
