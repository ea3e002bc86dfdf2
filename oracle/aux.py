"""Oracle for the image-space auxiliary terms of the training objective
(eq. 6 and eq. 17 name them without defining them).  TEST INFRASTRUCTURE
ONLY.  Plain numpy, FP64.

Readings used here (each term per view, summed over views, weights given by
the caller):
  transmittance concentration  L_Tc = 1/|P| sum_p A_p (1 - A_p)
      (A = 1 - T_K: zero when the final transmittance is 0 or 1, largest at
      1/2);
  distortion                   L_d  = 1/|P| sum_p dist_p
      (dist the per-pixel distortion channel of the renderer);
  depth-normal consistency     L_n  = 1/|I| sum_{p in I} (A_p - N_p . m_p)
      over the interior pixels I (1 <= x <= W-2, 1 <= y <= H-2), N the
      rendered normal channel and m the unit normal of the surface the
      depth channel describes: X_p = o + D_p d_p (d_p the pixel's unit ray),
      e_x = X(x+1, y) - X(x-1, y), e_y = X(x, y+1) - X(x, y-1),
      m = (e_y x e_x) / |e_y x e_x| (0 when the cross product vanishes),
      which faces the camera for a visible surface.  Since |N| <= A,
      L_n >= 0, with 0 when every blended voxel normal equals m.
  median depth-normal consistency (eq. 17's median-based variant)
                               L_nm = 1/|I| sum_{p in I} (A_p - N_p . m'_p)
      with m' the normal of the median-depth map M (the chord midpoint of the
      first hit after which the transmittance is at most 1/2, 0 where none
      is): the same stencil on M instead of D.  M is piecewise constant in
      the densities, so the term passes no depth gradient.
"""
from __future__ import annotations

import numpy as np

from . import pix_offsets


def pixel_dirs(cam) -> np.ndarray:
    """Unit world ray directions through the pixel centres, [H, W, 3]."""
    xs = (np.arange(cam.width) + 0.5 - cam.cx) / cam.fx
    ys = (np.arange(cam.height) + 0.5 - cam.cy) / cam.fy
    dc = np.stack(np.broadcast_arrays(xs[None, :], ys[:, None], np.ones((cam.height, 1))), -1)
    d = dc @ np.asarray(cam.R, np.float64)          # rows: R^T applied to each direction
    return d / np.linalg.norm(d, axis=-1, keepdims=True)


def depth_normals(depth: np.ndarray, cam):
    """Interior unit normals m [H-2, W-2, 3] of the depth map, with the
    cross products before normalisation and their lengths."""
    d = pixel_dirs(cam)
    X = np.asarray(cam.o, np.float64) + depth[..., None] * d
    ex = X[1:-1, 2:] - X[1:-1, :-2]
    ey = X[2:, 1:-1] - X[:-2, 1:-1]
    c = np.cross(ey, ex)
    ln = np.linalg.norm(c, axis=-1)
    m = np.where(ln[..., None] > 0, c / np.where(ln > 0, ln, 1.0)[..., None], 0.0)
    return m, c, ln, d


def aux_losses(depth, alpha, normal, dist, cams, lam_tc=1.0, lam_n=1.0, lam_d=1.0, mdepth=None,
               lam_nm=0.0):
    """Per-view losses [V, 4] (L_Tc, L_n, L_d, L_nm, each times its weight;
    L_nm is 0 without mdepth) and the gradients of their sum: g_alpha [P],
    g_depth [P], g_normal [3P] (rgb layout), g_dist [P]."""
    off = pix_offsets(cams)
    P = int(off[-1])
    depth, alpha, dist = (np.asarray(a, np.float64).ravel() for a in (depth, alpha, dist))
    normal = np.asarray(normal, np.float64).ravel()
    losses = np.zeros((len(cams), 4))
    if mdepth is not None:
        mdepth = np.asarray(mdepth, np.float64).ravel()
    g_alpha, g_depth, g_dist = np.zeros(P), np.zeros(P), np.zeros(P)
    g_normal = np.zeros(3 * P)
    for v, cam in enumerate(cams):
        H, W = cam.height, cam.width
        sl = slice(int(off[v]), int(off[v + 1]))
        A = alpha[sl].reshape(H, W)
        D = depth[sl].reshape(H, W)
        N = normal[3 * int(off[v]):3 * int(off[v + 1])].reshape(3, H, W).transpose(1, 2, 0)
        npx = H * W
        ga = lam_tc * (1.0 - 2.0 * A) / npx
        losses[v, 0] = lam_tc * float(np.sum(A * (1.0 - A))) / npx
        losses[v, 2] = lam_d * float(np.sum(dist[sl])) / npx
        g_dist[sl] = lam_d / npx
        gd = np.zeros((H, W))
        gn = np.zeros((H, W, 3))
        if H >= 3 and W >= 3:
            ni = (H - 2) * (W - 2)
            m, c, ln, dirs = depth_normals(D, cam)
            Ai, Ni = A[1:-1, 1:-1], N[1:-1, 1:-1]
            losses[v, 1] = lam_n * float(np.sum(Ai - np.sum(Ni * m, -1))) / ni
            ga[1:-1, 1:-1] += lam_n / ni
            gn[1:-1, 1:-1] = -lam_n * m / ni
            # through m = c / |c|, c = e_y x e_x, e_x, e_y differences of X = o + D d
            gm = -lam_n * Ni / ni
            lsafe = np.where(ln > 0, ln, 1.0)[..., None]
            gc = np.where(ln[..., None] > 0, (gm - m * np.sum(gm * m, -1, keepdims=True)) / lsafe, 0.0)
            ex = (np.asarray(cam.o) + D[1:-1, 2:, None] * dirs[1:-1, 2:]) - \
                 (np.asarray(cam.o) + D[1:-1, :-2, None] * dirs[1:-1, :-2])
            ey = (np.asarray(cam.o) + D[2:, 1:-1, None] * dirs[2:, 1:-1]) - \
                 (np.asarray(cam.o) + D[:-2, 1:-1, None] * dirs[:-2, 1:-1])
            gey = np.cross(ex, gc)      # d(ey x ex)/d ey applied to gc
            gex = np.cross(gc, ey)      # d(ey x ex)/d ex applied to gc
            gX = np.zeros((H, W, 3))
            gX[1:-1, 2:] += gex
            gX[1:-1, :-2] -= gex
            gX[2:, 1:-1] += gey
            gX[:-2, 1:-1] -= gey
            gd = np.sum(gX * pixel_dirs(cam), -1)
            if mdepth is not None:
                mm, _, _, _ = depth_normals(mdepth[sl].reshape(H, W), cam)
                losses[v, 3] = lam_nm * float(np.sum(Ai - np.sum(Ni * mm, -1))) / ni
                ga[1:-1, 1:-1] += lam_nm / ni
                gn[1:-1, 1:-1] += -lam_nm * mm / ni
        g_alpha[sl] = ga.ravel()
        g_depth[sl] = gd.ravel()
        g_normal[3 * int(off[v]):3 * int(off[v + 1])] = gn.transpose(2, 0, 1).ravel()
    return losses, g_alpha, g_depth, g_normal, g_dist
