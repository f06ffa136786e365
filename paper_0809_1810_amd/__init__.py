"""MI355X-native vortex-particle Fast Multipole Method (Cruz & Barba 2008).

The computation lives in the HIP library ``libvfmm.so`` (C ABI in
``include/vfmm.h``); this package is its thin Python binding.
"""
from .vfmm import (Batch, FP32, FP64, M2L_BF16, M2L_FP16, MAX_LEVELS, MAX_P, MLP_PARAMS, N_FEATURES,
                   PART_ALL, PART_FAR, PART_NEAR, PRECISIONS, MlpTrainer, Tree, VfmmError,
                   VfmmUnavailable, build_tree, direct_velocity, error_metrics, fmm_velocity,
                   header_symbols, lib, mlp_forward, fmm_velocity_oneshot, particle_stats, select_params,
                   selector_features, set_tuning, get_tuning, workspace_bytes,
                   direct_velocity_at, error_field, targets_workspace_bytes, NEAR_RADIUS_AUTO,
                   NEAR_RINGS_MAX, substitution_bound,
                   N_PHASES, PHASES)

__all__ = [
    "Batch", "FP32", "FP64", "M2L_BF16", "M2L_FP16", "MAX_LEVELS", "MAX_P", "MLP_PARAMS", "N_FEATURES",
    "PART_ALL", "PART_FAR", "PART_NEAR", "PRECISIONS", "MlpTrainer", "Tree", "VfmmError",
    "VfmmUnavailable", "build_tree", "direct_velocity", "error_metrics", "fmm_velocity",
    "header_symbols", "lib", "mlp_forward", "fmm_velocity_oneshot", "particle_stats", "select_params",
    "selector_features", "set_tuning", "get_tuning", "workspace_bytes",
    "direct_velocity_at", "error_field", "targets_workspace_bytes", "NEAR_RADIUS_AUTO",
    "NEAR_RINGS_MAX", "substitution_bound",
    "N_PHASES", "PHASES",
]
