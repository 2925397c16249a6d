"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This package holds no arithmetic of the reconstruction method itself: it draws
random phantom parameters, rasterises them onto voxel grids, draws random test
arrays, and names the workload presets (geometry scalars only).  Both the FP64
oracle (``oracle/``) and the HIP path (``paper_1904_13342_amd``) take their
inputs from here; neither imports the other.
"""
from .phantom import (
    random_ellipses,
    random_ellipsoids,
    rasterize_ellipses,
    rasterize_ellipsoids,
    random_gaussians,
    rasterize_gaussians,
    disk,
    sphere,
    grid_axes,
)
from .configs import CONFIGS, config, GeometrySpec
from .rng import random_array
from .trajectory import perturbed_poses, pose_matrices, pixel_positions

__all__ = [
    "random_ellipses",
    "random_ellipsoids",
    "rasterize_ellipses",
    "rasterize_ellipsoids",
    "random_gaussians",
    "rasterize_gaussians",
    "disk",
    "sphere",
    "grid_axes",
    "CONFIGS",
    "config",
    "GeometrySpec",
    "random_array",
    "perturbed_poses",
    "pose_matrices",
    "pixel_positions",
]
