"""Oracle for grid-point density storage with a density activation (the
SVRaster-style parameterisation the paper starts from, Sec. III "Loss
Optimization" context of eq. 6).  TEST INFRASTRUCTURE ONLY.

Reading used here (the paper does not define the storage or the activation):
  raw values live on shared grid points; corner c of voxel v takes
  act(raw[corner_idx[c][v]]), or 0 when the index lies outside
  [0, n_grid); act is the identity, softplus log(1 + e^x) or exp, applied to
  each grid value before the trilinear interpolation, so the density inside
  a voxel stays trilinear and its chord integral exact.  In the dense layout
  (one raw value per voxel corner) the same activation applies per corner.
The gradient of a loss with respect to a raw grid value is the sum, over the
corners that read it, of the corner-value gradient (the rasterizer's adjoint,
eq. 2-4) times act'(raw).  Everything here is FP64.
"""
from __future__ import annotations

import numpy as np

ACT_NONE, ACT_SOFTPLUS, ACT_EXP = 0, 1, 2


def activate(x, act):
    x = np.asarray(x, dtype=np.float64)
    if act == ACT_SOFTPLUS:
        return np.logaddexp(0.0, x)
    if act == ACT_EXP:
        return np.exp(x)
    return x.copy()


def activate_grad(x, act):
    x = np.asarray(x, dtype=np.float64)
    if act == ACT_SOFTPLUS:
        return 1.0 / (1.0 + np.exp(-x))
    if act == ACT_EXP:
        return np.exp(x)
    return np.ones_like(x)


def corner_values(grid, corner_idx, act):
    """[8][N] corner densities read from the grid."""
    grid = np.asarray(grid, dtype=np.float64)
    idx = np.asarray(corner_idx, dtype=np.int64)
    ok = (idx >= 0) & (idx < grid.shape[0])
    out = np.zeros(idx.shape, dtype=np.float64)
    out[ok] = activate(grid[idx[ok]], act)
    return out


def grid_gradient(d_corner, grid, corner_idx, act):
    """Scatter of the corner-value gradient [8][N] onto the raw grid values."""
    grid = np.asarray(grid, dtype=np.float64)
    idx = np.asarray(corner_idx, dtype=np.int64)
    ok = (idx >= 0) & (idx < grid.shape[0])
    d = np.zeros(grid.shape[0], dtype=np.float64)
    np.add.at(d, idx[ok], np.asarray(d_corner, dtype=np.float64)[ok] * activate_grad(grid[idx[ok]], act))
    return d


def with_corners(scene, corners):
    """The same leaves with the given [8][N] corner densities."""
    import dataclasses
    return dataclasses.replace(scene, density=np.asarray(corners, dtype=np.float64))
