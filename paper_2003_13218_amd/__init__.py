"""Periodic FMM for charged systems neutralised by a uniform background charge
(arXiv:2003.13218) on AMD Instinct MI355X (gfx950).

The GPU library is ``libfmm.so`` (C ABI in ``include/fmm.h``); ``binding``
is its thin Python wrapper.  Importing this package does not load the library;
``binding.load()`` does, and raises if it has not been built.
"""
from . import binding  # noqa: F401
from .binding import (FMM_FP64, FMM_MIXED, FMM_MIXED_BF16_M2L, FMM_MIXED_SPLIT16_M2L, FMM_BOUNDARY_CONDUCTING,  # noqa: F401
                      FMM_BOUNDARY_VACUUM, FMM_UV_SYMMETRIC, FMM_UV_SPARSE, FMM_UV_SWAP, FmmError, Plan, fmm_bin, fmm_destroy,  # noqa: F401
                      fmm_energy_forces, fmm_last_error, fmm_lattice_tensor, fmm_plan,
                      fmm_plan_config, fmm_potential_parts, fmm_profile, fmm_profile_read,
                      fmm_solute_solvent_energy, fmm_version, fmm_plan_batch, fmm_energy_forces_batch,
                      fmm_solute_solvent_energy_batch, fmm_autotune_batch, fmm_batch_levels,
                      fmm_lambda_energy, fmm_lambda_energy_batch, fmm_plan_options,
                      fmm_plan_softcore, fmm_plan_info, fmm_plan_tuning,
                      fmm_energy_forces_noalloc, fmm_batch_set_tuning, fmm_autotune_batch_cached)
