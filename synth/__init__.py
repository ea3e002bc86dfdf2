"""Seeded synthetic inputs shared by the HIP path, the oracle, the tests and the bench.

This package only draws inputs: octree leaf sets, corner densities, SH
coefficients, pinhole cameras and smooth target images.  It contains none of
the rasterizer's arithmetic (no projection, binning, compositing, loss or
gradient), so the oracle and the HIP path can both consume it without sharing
any of the method.
"""
from .scenes import (  # noqa: F401
    Scene, Camera, CONFIGS, make_config, make_scene_grid, make_scene_shell,
    make_cameras_single, make_cameras_ring, make_cameras_hemisphere,
    make_target, scene_subset, config_seed, grid_points,
)
