"""Oracle for the low-frequency-aware photometric term (Sec. IV-B, eq. 7-10),
FP64 numpy.  TEST INFRASTRUCTURE ONLY.

  grey(p)   = mean of the target's three channels
  g(p)      = |Sobel(grey)| with replicated borders (3x3 kernels)
  g99       = nearest-rank 99th percentile of g over the view
  s(p)      = min(1, g / g99)  (0 everywhere when g99 = 0)
  form 0    : w = (eps + 1 - s)^gamma                       (eq. 7)
  form 1    : w = (1 + g / g99)^-gamma                      (the configured ramp form)
  w~        = w / mean(w)                                   (eq. 8)
  L_view    = mean_p w~(p) * mean_ch |C - I|                (eq. 10, rho = L1)
  dL/dC     = w~ * sign(C - I) / (3 |P|),   sign(0) = 0
  gamma(t)  = piecewise-linear ramp                         (eq. 9)
"""
from __future__ import annotations

import math

import numpy as np


def nearest_rank(values: np.ndarray, q: float):
    """Smallest x with empirical CDF F(x) >= q: the ceil(q n)-th smallest."""
    v = np.sort(np.asarray(values).ravel())
    n = v.shape[0]
    r = int(math.ceil(q * n))
    r = min(max(r, 1), n)
    return v[r - 1]


def sobel_magnitude(grey: np.ndarray) -> np.ndarray:
    p = np.pad(np.asarray(grey, dtype=np.float64), 1, mode="edge")
    gx = (p[:-2, 2:] + 2.0 * p[1:-1, 2:] + p[2:, 2:]) - (p[:-2, :-2] + 2.0 * p[1:-1, :-2] + p[2:, :-2])
    gy = (p[2:, :-2] + 2.0 * p[2:, 1:-1] + p[2:, 2:]) - (p[:-2, :-2] + 2.0 * p[:-2, 1:-1] + p[:-2, 2:])
    return np.sqrt(gx * gx + gy * gy)


def lf_weight(target: np.ndarray, gamma: float, form: int = 0, eps: float = 1e-3,
              q: float = 0.99) -> np.ndarray:
    """Mean-normalised inverse-Sobel weight of one view; target [3, H, W]."""
    grey = np.asarray(target, dtype=np.float64).mean(axis=0)
    g = sobel_magnitude(grey)
    g99 = nearest_rank(g, q)
    ratio = g / g99 if g99 > 0 else np.zeros_like(g)
    if form == 0:
        s = np.minimum(1.0, ratio)
        w = (eps + 1.0 - s) ** gamma
    else:
        w = (1.0 + ratio) ** (-gamma)
    return w / w.mean()


def l1_loss_grad(rgb: np.ndarray, target: np.ndarray, weight: np.ndarray):
    """Weighted L1 of one view: (loss, dL/drgb [3, H, W])."""
    r = np.asarray(rgb, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    npix = weight.size
    loss = float((weight * np.abs(r).mean(axis=0)).sum() / npix)
    grad = weight[None] * np.sign(r) / (3.0 * npix)
    return loss, grad


def gamma_schedule(t: float, total: float, t0_frac: float = 0.3, t1_frac: float = 0.6,
                   gamma_max: float = 0.6) -> float:
    t0, t1 = t0_frac * total, t1_frac * total
    if t < t0:
        return 0.0
    if t < t1:
        return gamma_max * (t - t0) / (t1 - t0)
    return gamma_max
