"""Seeded synthetic inputs for the extrapolated-regularization Stokes layer potentials.

This package only *generates inputs*: surface quadratures, target sets and smooth vector densities.
It contains none of the layer-potential arithmetic (kernels, smoothing, extrapolation), so both the
CPU oracle and the GPU library consume its arrays without sharing any of the method's code.
"""
from .surface import (Surface, ellipsoid_quadrature, ellipsoid_normal, ellipsoid_project,
                      closest_point_ellipsoid, ellipsoid_area, sphere_quadrature)
from .targets import Targets, on_surface_targets, near_targets, grid_targets_outside, concat_targets
from .density import harmonic_coeffs, harmonic_field
from .configs import build_config, CONFIGS, two_spheres, rigid_motion, two_drops, drop_force
from .warmstart import mlp_init, warmstart_samples, warmstart_dataset, warmstart_unit_dataset, GAP_RANGE

__all__ = [
    "Surface", "ellipsoid_quadrature", "ellipsoid_normal", "ellipsoid_project", "closest_point_ellipsoid",
    "ellipsoid_area", "sphere_quadrature", "Targets", "on_surface_targets", "near_targets",
    "grid_targets_outside", "concat_targets", "harmonic_coeffs", "harmonic_field", "build_config", "CONFIGS",
    "two_spheres", "rigid_motion", "two_drops", "drop_force", "mlp_init", "warmstart_samples", "warmstart_dataset", "warmstart_unit_dataset", "GAP_RANGE",
]
