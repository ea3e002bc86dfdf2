"""Oracle for the pruning stability guards (Sec. IV-C, guards i-iii), applied
at each adaptation step on top of the per-bin quantile decision (eq. 11-12).
TEST INFRASTRUCTURE ONLY.

The paper names the three guards but fixes neither the inside score nor any
constant.  Reading used here (each constant is a caller parameter):
  x_v  = 1 if w_max_v > tau_{bin(v)}, else 0      (the voxel survives the
         per-bin quantile test of eq. 12: the inside score)
  i.   m_v <- (1 - alpha) m_v + alpha x_v          (exponential moving average)
       s_v <- out if m_v < m_low, in if m_v > m_high, else unchanged
  ii.  keep-halo: protected_v = (delta_v finite and h_v < rho delta_v)
       or w_max_v >= w_keep, with h_v the half edge and delta_v the inter-ray
       spacing at the voxel centre (the footprint of eq. 13-14)
  iii. candidates = out and not protected; with cap = floor(cap_frac n)
       (double), the first min(cap, #candidates) candidates in the order
       (m_v, v) are pruned.  m is ordered by its binary32 value, -0 before +0.
Every step that decides an integer is binary32, one rounded operation at a
time in the order written:
  m  = fl( fl(fl(1 - alpha) m) + fl(alpha x) )
  h  = fl(0.5 e),  e = root_size 2^-l
  rd = fl(rho delta)
"""
from __future__ import annotations

import math

import numpy as np

from .quantile import depth_proxy

f32 = np.float32


def order_key(m: np.ndarray) -> np.ndarray:
    """uint32 whose unsigned order is the binary32 order of m (-0 < +0)."""
    u = np.asarray(m, dtype=f32).view(np.uint32)
    return np.where(u & np.uint32(0x80000000), ~u, u | np.uint32(0x80000000)).astype(np.uint32)


def ema_update(ema, x, alpha):
    a = f32(alpha)
    return (f32(f32(1.0) - a) * np.asarray(ema, dtype=f32) + a * np.asarray(x, dtype=f32)).astype(f32)


def hysteresis(m, state, m_low, m_high):
    s = np.asarray(state, dtype=np.uint8)
    return np.where(m < f32(m_low), 0, np.where(m > f32(m_high), 1, s)).astype(np.uint8)


def keep_halo(scene, delta, wmax, rho, w_keep):
    e = np.ldexp(f32(scene.root_size), -scene.level.astype(np.int32)).astype(f32)
    h = (f32(0.5) * e).astype(f32)
    fin = np.isfinite(delta)
    rd = np.where(fin, f32(rho) * np.where(fin, delta, f32(0.0)), f32(0.0)).astype(f32)
    return (fin & (h < rd)) | (np.asarray(wmax, dtype=f32) >= f32(w_keep))


def capped_prune(cand, m, cap_frac):
    n = cand.shape[0]
    cap = int(math.floor(float(cap_frac) * float(n)))
    idx = np.nonzero(cand)[0]
    order = np.lexsort((idx, order_key(m[idx])))   # last key is primary
    prune = np.zeros(n, dtype=np.uint8)
    prune[idx[order[:cap]]] = 1
    return prune


def guard_step(scene, cams, wmax, bins, tau, ema, state, alpha=0.3, m_low=0.3, m_high=0.7,
               rho=0.25, w_keep=0.5, cap_frac=0.05):
    """One adaptation step.  Returns (prune u8 [n], ema f32 [n], state u8 [n])."""
    wmax = np.asarray(wmax, dtype=f32)
    tau = np.asarray(tau, dtype=f32)
    x = (wmax > tau[np.asarray(bins, dtype=np.int64)]).astype(np.uint8)
    m = ema_update(ema, x, alpha)
    s = hysteresis(m, state, m_low, m_high)
    prot = keep_halo(scene, depth_proxy(scene, cams), wmax, rho, w_keep)
    cand = (s == 0) & ~prot
    return capped_prune(cand, m, cap_frac), m, s
