"""MI355X-native vielbein lattice Boltzmann (vLBM) on the sphere.

The compute path is ``libvlbm.so`` (HIP, gfx950) behind the C ABI of
``include/vlbm.h``; :mod:`paper_2504_15574_amd.vlbm` is its ctypes binding.
"""
from .vlbm import (  # noqa: F401
    ABI_VERSION, LIB_PATH, SIGNATURES, STORAGE, Ensemble, Solver, VlbmError, load, make_params,
    vlbm_create, vlbm_destroy, vlbm_diagnostics, vlbm_get_populations, vlbm_init_fields,
    vlbm_moments, vlbm_set_populations, vlbm_stage_launches, vlbm_step, vlbm_suggest_dt,
    vlbm_vorticity, vlbm_workspace_bytes, vlbm_step_batch, vlbm_graph_create, vlbm_graph_launch,
    vlbm_graph_destroy, vlbm_quadrature_f32, vlbm_correct_moments, vlbm_set_tile_shape,
    vlbm_step_batch_persistent, vlbm_set_barrier_spin_limit, vlbm_graph_create_persistent,
    vlbm_graph_check, vlbm_diagnostics_static,
)
