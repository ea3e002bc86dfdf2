"""Oracle for footprint-eligible, priority-driven subdivision (Sec. IV-D,
eq. 13-16) and the 8-way split.  TEST INFRASTRUCTURE ONLY.

Reading used here (the paper leaves the usefulness score, the depth used per
voxel and the child initialisation open):
  delta_v  = inter-ray spacing at the voxel centre (the footprint; the same
             binary32 definition as the depth-quantile oracle), h_v = e_v / 2
  eligible = l_v < 12 and delta_v finite and h_v > kappa delta_v     (eq. 13)
  z~_v     = clip((delta_v - z5) / (z95 - z5), 0, 1) with the caller's running
             percentiles (z5, z95) of delta (eq. 14; the same special cases as
             the quantile: +inf -> 1, z95 <= z5 or z95 = +inf -> 0)
  P'_v     = P_v (1 + beta z~_v), P_v the caller's usefulness score (eq. 15-16)
  split    = the first min(max_splits, #candidates) eligible voxels with
             P'_v > 0 in the order (P'_v descending, v ascending)
  children = the 8 cells of the next level (child c = x + 2y + 4z bits, ijk
             2 ijk + bits); a child's corner densities are the parent's
             trilinear field at that corner, built from midpoints
             mid(a, b) = 0.5 a + 0.5 b taken along x, then y, then z (exact
             refinement: the density field is unchanged); SH coefficients
             are copied.  The refined set keeps the input order, each split
             voxel replaced in place by its 8 children; a split flag on a
             leaf at the finest level is ignored.
Binary32, one rounded operation at a time in the order written, wherever the
result decides an integer or is stored.
"""
from __future__ import annotations

import numpy as np

from .guard import order_key
from .quantile import depth_proxy, nearest_rank_index

f32 = np.float32
L_MAX = 12


def footprint_range(scene, cams):
    """Nearest-rank 5th and 95th percentiles of delta over all voxels."""
    d = np.sort(depth_proxy(scene, cams))
    n = d.shape[0]
    if n == 0:
        return f32(0.0), f32(0.0)
    return f32(d[nearest_rank_index(n, 0.05)]), f32(d[nearest_rank_index(n, 0.95)])


def normalised_depth(delta, z5, z95):
    zt = np.zeros(delta.shape[0], dtype=f32)
    fin = np.isfinite(delta)
    if np.isfinite(z95) and z95 > z5:
        den = f32(f32(z95) - f32(z5))
        zt[fin] = np.clip((delta[fin] - f32(z5)) / den, f32(0.0), f32(1.0))
    zt[~fin] = f32(1.0)
    return zt


def select(scene, cams, score, z5, z95, kappa=1.0, beta=0.2, max_splits=1000):
    """Returns (split u8 [n], priority f32 [n], eligible bool [n])."""
    delta = depth_proxy(scene, cams)
    e = np.ldexp(f32(scene.root_size), -scene.level.astype(np.int32)).astype(f32)
    h = (f32(0.5) * e).astype(f32)
    fin = np.isfinite(delta)
    kd = np.where(fin, f32(kappa) * np.where(fin, delta, f32(0.0)), f32(0.0)).astype(f32)
    elig = (scene.level.astype(np.int32) < L_MAX) & fin & (h > kd)
    zt = normalised_depth(delta, z5, z95)
    bias = (f32(1.0) + f32(beta) * zt).astype(f32)
    prio = (np.asarray(score, dtype=f32) * bias).astype(f32)
    cand = elig & (prio > f32(0.0))
    idx = np.nonzero(cand)[0]
    key = ~order_key(prio[idx])          # ascending key = descending priority
    order = np.lexsort((idx, key))
    split = np.zeros(scene.n, dtype=np.uint8)
    split[idx[order[:int(max_splits)]]] = 1
    return split, prio, elig


def _mid(a, b):
    return (f32(0.5) * a + f32(0.5) * b).astype(f32)


def child_densities(dens):
    """dens f32 [8][m] parent corners -> [8 children][8 corners][m]."""
    out = np.empty((8, 8, dens.shape[1]), dtype=f32)
    for ch in range(8):
        b = ((ch >> 0) & 1, (ch >> 1) & 1, (ch >> 2) & 1)
        for co in range(8):
            c = ((co >> 0) & 1, (co >> 1) & 1, (co >> 2) & 1)
            u2 = [b[a] + c[a] for a in range(3)]        # 2u in {0, 1, 2}
            # along x: a value per (y, z) corner pair of the parent
            fx = {}
            for y in (0, 1):
                for z in (0, 1):
                    s0, s1 = dens[0 + 2 * y + 4 * z], dens[1 + 2 * y + 4 * z]
                    fx[(y, z)] = s0 if u2[0] == 0 else (s1 if u2[0] == 2 else _mid(s0, s1))
            fy = {}
            for z in (0, 1):
                a0, a1 = fx[(0, z)], fx[(1, z)]
                fy[z] = a0 if u2[1] == 0 else (a1 if u2[1] == 2 else _mid(a0, a1))
            out[ch, co] = fy[0] if u2[2] == 0 else (fy[1] if u2[2] == 2 else _mid(fy[0], fy[1]))
    return out


def apply_split(scene, split):
    """The refined voxel set (same Scene type), input order kept."""
    from synth.scenes import Scene
    split = np.asarray(split, dtype=bool) & (scene.level.astype(np.int32) < L_MAX)   # finest: no children
    n = scene.n
    reps = np.where(split, 8, 1)
    m = int(reps.sum())
    src = np.repeat(np.arange(n), reps)
    first = np.concatenate([[0], np.cumsum(reps)[:-1]])
    kid = np.arange(m) - np.repeat(first, reps)          # child index (0 for unsplit)
    is_child = split[src]
    bits = [(kid >> a) & 1 for a in range(3)]
    ijk = np.empty((3, m), dtype=np.uint16)
    for a in range(3):
        base = scene.ijk[a][src].astype(np.int64)
        ijk[a] = np.where(is_child, 2 * base + bits[a], base).astype(np.uint16)
    level = np.where(is_child, scene.level[src].astype(np.int32) + 1, scene.level[src]).astype(np.uint8)
    dens = scene.density[:, src].astype(f32).copy()
    if split.any():
        kids = child_densities(scene.density[:, split].astype(f32))   # [8][8][k]
        rows = np.nonzero(is_child)[0]
        k_of = np.cumsum(split) - 1                                   # parent -> split rank
        ks = k_of[src[rows]]
        dens[:, rows] = kids[kid[rows], :, ks].T
    sh = scene.sh[:, src].astype(f32)
    return Scene(root_min=scene.root_min.copy(), root_size=scene.root_size, ijk=ijk, level=level,
                 density=dens, sh=sh, sh_degree=scene.sh_degree)
