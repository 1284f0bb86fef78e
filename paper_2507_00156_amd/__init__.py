"""Extrapolated-regularization Stokes single/double-layer sums on MI355X (gfx950).

The compute path is libstokesreg.so (hand-written HIP kernels behind the C ABI of
include/stokesreg.h); `binding` marshals torch tensors into it and `Evaluator` is a small
convenience wrapper.  Nothing here computes the method on the CPU.
"""
from .binding import (EXPORTS, LIB_PATH, SR_DIRECT, SR_DL, SR_FP64, SR_MIXED, SR_SL, SR_TREE, SR_HOST, SR_ENEAR,
                      SrError, SrParams, sr_eval_far, sr_check, sr_max_targets, sr_near_table,
                      load_library, sr_create, sr_default_params, sr_destroy, sr_eval, sr_set_density,
                      sr_set_params, sr_set_surface, sr_version, sr_set_profiling, sr_get_profile,
                      SR_PHASE_FAR, SR_PHASE_NEAR, sr_rigid_create, sr_rigid_destroy, sr_rigid_set_params,
                      sr_rigid_set_spheres, sr_rigid_rhs, sr_rigid_matvec, sr_rigid_solve, sr_rigid_velocity,
                      sr_rigid_solve_refined, sr_mlp_gemm_test, sr_mlp_num_params)
from .evaluator import Evaluator, RigidSpheres, Prolongation, WarmStartNet

__all__ = ["EXPORTS", "LIB_PATH", "SR_DIRECT", "SR_DL", "SR_FP64", "SR_MIXED", "SR_SL", "SR_TREE", "SR_HOST",
           "SR_ENEAR", "sr_eval_far", "sr_check", "sr_max_targets", "sr_near_table", "SrError",
           "SrParams", "load_library", "sr_create", "sr_default_params", "sr_destroy", "sr_eval", "sr_set_density",
           "sr_set_params", "sr_set_surface", "sr_version", "Evaluator", "RigidSpheres", "sr_set_profiling", "sr_get_profile",
           "SR_PHASE_FAR", "SR_PHASE_NEAR", "sr_rigid_create", "sr_rigid_destroy", "sr_rigid_set_params",
           "sr_rigid_set_spheres", "sr_rigid_rhs", "sr_rigid_matvec", "sr_rigid_solve", "sr_rigid_velocity",
           "sr_rigid_solve_refined", "sr_mlp_gemm_test", "sr_mlp_num_params", "Prolongation", "WarmStartNet"]
