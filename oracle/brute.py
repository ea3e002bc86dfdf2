"""Brute-force volume-rendering integral along one ray (TEST INFRASTRUCTURE).

Independent of the chord/polynomial machinery of the oracle: the ray is
sampled at the midpoints of n_steps equal steps; at each sample the density
is found by locating the containing voxel by exhaustive search and
interpolating its corner values trilinearly; colour is the voxel's constant
(degree-0) colour.  The continuous integral C = int T(t) sigma(t) c(t) dt,
T(t) = exp(-int_0^t sigma), is accumulated step by step, so C and 1 - T(inf)
converge (second order in the step) to the values of eq. 2-4 for piecewise
trilinear density.
"""
from __future__ import annotations

import numpy as np


def integrate_ray(scene, o, d, t_max, n_steps=200_000):
    o = np.asarray(o, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    d = d / np.linalg.norm(d)
    dt = t_max / n_steps
    t = (np.arange(n_steps) + 0.5) * dt
    p = o[None, :] + t[:, None] * d[None, :]
    sigma = np.zeros(n_steps)
    col = np.zeros((n_steps, 3))
    e_all = scene.root_size * np.exp2(-scene.level.astype(np.float64))
    b_all = scene.root_min[:, None].astype(np.float64) + scene.ijk.astype(np.float64) * e_all
    for v in range(scene.n):
        e = e_all[v]
        b = b_all[:, v]
        inside = np.all((p >= b) & (p < b + e), axis=1)
        if not inside.any():
            continue
        u = (p[inside] - b) / e
        s = np.zeros(u.shape[0])
        for c in range(8):
            wgt = np.ones(u.shape[0])
            for a in range(3):
                wgt *= u[:, a] if (c >> a) & 1 else 1.0 - u[:, a]
            s += scene.density[c, v] * wgt
        sigma[inside] = s
        col[inside] = np.maximum(scene.sh[0:3, v].astype(np.float64), 0.0)
    od = sigma * dt
    T_before = np.exp(-np.concatenate([[0.0], np.cumsum(od)[:-1]]))
    w = T_before * -np.expm1(-od)
    C = (w[:, None] * col).sum(axis=0)
    T_end = float(np.exp(-od.sum()))
    return C, 1.0 - T_end
