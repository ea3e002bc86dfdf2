"""Oracle for depth-aware quantile pruning (Sec. IV-C, eq. 11-12 and 14).
TEST INFRASTRUCTURE ONLY.

Every step whose floating-point result decides an integer (a voxel's bin) is
taken in binary32, one rounded operation at a time in the order written, so
that the bin of each voxel is defined exactly:
  x_v       = b_v + 0.5 e_v                                 (voxel centre)
  z_c       = (R20 q0 + R21 q1) + R22 q2,  q = x_v - o
  delta_v   = min over views with z_c > 0 of z_c / f_x      (inter-ray spacing,
              the paper's depth proxy); +inf if no view sees it in front
  p5, p95   = nearest-rank 5th / 95th percentiles of delta over all voxels
  z~        = clip((delta - p5) / (p95 - p5), 0, 1)          (eq. 14)
              (+inf -> 1; p95 <= p5 or p95 = +inf -> 0 for finite delta)
  bin       = min(B - 1, floor(B z~))
  tau_b     = F_b^{-1}(q): the ceil(q |V_b|)-th smallest w_max of bin b
              (eq. 11-12; rank taken in double); -inf for an empty bin
  prune_v   = w_max_v <= tau_{bin(v)}
"""
from __future__ import annotations

import math

import numpy as np

f32 = np.float32


def depth_proxy(scene, cams) -> np.ndarray:
    n = scene.n
    e = np.ldexp(f32(scene.root_size), -scene.level.astype(np.int32)).astype(f32)
    b = [f32(scene.root_min[a]) + scene.ijk[a].astype(f32) * e for a in range(3)]
    x = [b[a] + f32(0.5) * e for a in range(3)]
    delta = np.full(n, np.inf, dtype=f32)
    for c in cams:
        R = np.asarray(c.R, dtype=f32)
        q = [x[a] - f32(c.o[a]) for a in range(3)]
        z = (R[2, 0] * q[0] + R[2, 1] * q[1]) + R[2, 2] * q[2]
        d = z / f32(c.fx)
        ok = z > f32(0.0)
        delta = np.where(ok, np.minimum(delta, d), delta).astype(f32)
    return delta


def nearest_rank_index(n: int, q: float) -> int:
    r = int(math.ceil(float(q) * float(n)))
    return min(max(r, 1), n) - 1


def depth_bins(delta: np.ndarray, n_bins: int):
    n = delta.shape[0]
    s = np.sort(delta)
    p5 = s[nearest_rank_index(n, 0.05)]
    p95 = s[nearest_rank_index(n, 0.95)]
    bins = np.zeros(n, dtype=np.int32)
    fin = np.isfinite(delta)
    if np.isfinite(p95) and p95 > p5:
        den = f32(p95 - p5)
        zt = (delta[fin] - f32(p5)) / den
        zt = np.clip(zt, f32(0.0), f32(1.0)).astype(f32)
        bins[fin] = np.minimum(n_bins - 1, np.floor(f32(n_bins) * zt).astype(np.int32))
    bins[~fin] = n_bins - 1
    return bins, f32(p5), f32(p95)


def quantile_cutoffs(wmax: np.ndarray, bins: np.ndarray, n_bins: int, q: float):
    wmax = np.asarray(wmax, dtype=f32)
    tau = np.full(n_bins, -np.inf, dtype=f32)
    for b in range(n_bins):
        vals = np.sort(wmax[bins == b])
        if vals.shape[0] == 0:
            continue
        tau[b] = vals[nearest_rank_index(vals.shape[0], q)]
    prune = (wmax <= tau[bins]).astype(np.uint8)
    return tau, prune


def depth_quantile(scene, cams, wmax, n_bins=16, q=0.1):
    delta = depth_proxy(scene, cams)
    bins, p5, p95 = depth_bins(delta, n_bins)
    tau, prune = quantile_cutoffs(wmax, bins, n_bins, q)
    return dict(delta=delta, bins=bins, p5=p5, p95=p95, tau=tau, prune=prune)
