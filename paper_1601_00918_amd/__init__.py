"""MI355X two-component lattice Boltzmann library (Python binding).

The binding marshals arguments to the C ABI of ``include/lbm.h``; every step of
the computation runs in the HIP kernels of ``liblbm.so``.  PyTorch provides the
device workspace and the stream.  Functions keep the ABI's names:

    lbm_required_bytes, lbm_init, lbm_step, lbm_time, lbm_set_fluid,
    lbm_moments, lbm_monitors, lbm_get_populations, lbm_fluid_mask, lbm_set_tiling,
    lbm_get_tiling, lbm_set_active, lbm_snapshot_save, lbm_snapshot_restore,
    lbm_cp_required_bytes, lbm_critical_pressure, lbm_cp_drive, lbm_destroy

``Simulation`` bundles a context with the torch workspace that backs it.
The D3Q19 tube and box (include/lbm3d.h) are in ``binding3d`` (``Simulation3D``,
``lbm3d_*``, ``lbm3d_critical_pressure``); the surrogate network's kernels
(include/lbm_mlp.h) in ``mlp``.
"""
from .binding import (Simulation, cp_options, cp_problem, fluid_struct, geom_struct,
                      init_struct, lbm_cp_drive, lbm_cp_required_bytes, lbm_critical_pressure,
                      lbm_destroy, lbm_fluid_mask, lbm_get_populations, lbm_get_tiling,
                      lbm_init, lbm_moments, lbm_monitors, lbm_required_bytes, lbm_set_active,
                      lbm_set_fluid, lbm_set_tiling, lbm_snapshot_restore, lbm_snapshot_save,
                      lbm_step, lbm_time, lbm_version)

__all__ = [
    "Simulation", "geom_struct", "fluid_struct", "init_struct", "lbm_destroy",
    "lbm_fluid_mask", "lbm_get_populations", "lbm_init", "lbm_moments", "lbm_monitors",
    "lbm_required_bytes", "lbm_set_fluid", "lbm_step", "lbm_time", "lbm_version",
    "lbm_set_tiling", "lbm_get_tiling", "lbm_set_active", "lbm_snapshot_save",
    "lbm_snapshot_restore", "cp_options", "cp_problem", "lbm_cp_required_bytes",
    "lbm_critical_pressure", "lbm_cp_drive",
]
