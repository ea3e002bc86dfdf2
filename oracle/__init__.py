"""Oracle: a plain, slow, FP64 CPU implementation of the LiteVoxel rasterizer
hot path.  TEST INFRASTRUCTURE ONLY -- imported by the tests, by the smoke
check and by the benchmark's CPU-baseline leg, never by the product path, and
sharing no code with the HIP library.

Parts and the passages they follow:
  raster_ref.cpp  rays, voxels, compositing, w_max           Sec. III, eq. 1-5
                  analytic adjoint of eq. 2-4 (ref_backward)
                  binary32 binning + visibility code (key path)
  raster_ref.cpp  auxiliary channels (ref_render_aux,           eq. 6, 17 (named
                  ref_backward_aux): distortion, normal;       terms; readings
                  median depth (ref_median_depth)              in the file)
  aux.py          transmittance concentration, depth-normal
                  consistency, distortion mean (image terms)   eq. 6, 17
  loss.py         inverse-Sobel weight, mean normalisation,
                  gamma(t) ramp, weighted L1 and its gradient  Sec. IV-B, eq. 7-10
  quantile.py     depth proxy, eq. 14 normalisation, per-bin
                  quantile cutoff and prune mask             Sec. IV-C, eq. 11-12, 14
  brute.py        per-ray numerical integration of the continuous
                  volume-rendering integral (an independent pin)

Pixel layout: views are packed in order; the global pixel index of (x, y) in
view v is off[v] + y*W + x.  RGB images are [3, H, W] per view.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "raster_ref.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-shared", "-fPIC", _SRC, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, f64, f32 = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_float
        L.ref_sh_basis.argtypes = [i64, i32, P, P]
        L.ref_render.argtypes = [i64, i32, P, f64, P, P, P, P, i32, P, P, P, P, i64,
                                 P, P, P, P, P, i32]
        L.ref_render.restype = i32
        L.ref_trace_pixel.argtypes = [i64, i32, P, f64, P, P, P, P, P, P, i32, i32, i32,
                                      P, P, P, P, P, P]
        L.ref_trace_pixel.restype = i32
        L.ref_backward.argtypes = [i64, i32, P, f64, P, P, P, P, i32, P, P, P, P, i64,
                                   P, P, P, P, P, i32]
        L.ref_backward.restype = i32
        L.ref_render_aux.argtypes = [i64, i32, P, f64, P, P, P, P, i32, P, P, P,
                                     P, P, P, P, P, P, i32]
        L.ref_render_aux.restype = i32
        L.ref_backward_aux.argtypes = [i64, i32, P, f64, P, P, P, P, i32, P, P, P,
                                       P, P, P, P, P, P, P, i32]
        L.ref_backward_aux.restype = i32
        L.ref_median_depth.argtypes = [i64, i32, P, f64, P, P, P, P, i32, P, P, f64, P, i32]
        L.ref_median_depth.restype = i32
        L.ref_footprint_pixels.argtypes = [i64, P, f64, P, P, i32, P, P, P, i64, P, i64]
        L.ref_footprint_pixels.restype = i64
        L.ref_voxel_colours.argtypes = [i64, i32, P, f64, P, P, P, i32, P, P, P, P]
        L.ref_voxel_colours.restype = i32
        L.ref_project_keys.argtypes = [i64, P, f32, P, P, i32, P, P, f32, P, P, P]
        L.ref_project_keys.restype = i32
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


# ---------------------------------------------------------------- marshalling

class _SceneArrays:
    def __init__(self, scene):
        self.n = scene.n
        self.deg = scene.sh_degree
        self.root_min = np.ascontiguousarray(scene.root_min, dtype=np.float32)
        self.root_size = float(scene.root_size)
        self.ijk = np.ascontiguousarray(scene.ijk, dtype=np.uint16)
        self.level = np.ascontiguousarray(scene.level, dtype=np.uint8)
        self.density = np.ascontiguousarray(scene.density, dtype=np.float64)
        self.sh = np.ascontiguousarray(scene.sh, dtype=np.float64)

    def args(self):
        return (self.n, self.deg, _p(self.root_min), self.root_size, _p(self.ijk),
                _p(self.level), _p(self.density), _p(self.sh))


def cams_arrays(cams):
    c = np.zeros((len(cams), 17), dtype=np.float32)
    wh = np.zeros((len(cams), 2), dtype=np.int32)
    for i, cam in enumerate(cams):
        c[i, 0:9] = np.asarray(cam.R, dtype=np.float32).ravel()
        c[i, 9:12] = cam.o
        c[i, 12:16] = [cam.fx, cam.fy, cam.cx, cam.cy]
        wh[i] = [cam.width, cam.height]
    return c, wh


def pix_offsets(cams):
    off = np.zeros(len(cams) + 1, dtype=np.int64)
    for i, c in enumerate(cams):
        off[i + 1] = off[i] + c.width * c.height
    return off


def split_views(flat_rgb, cams):
    """Flat [3*P] rgb buffer -> list of [3, H, W] views."""
    off = pix_offsets(cams)
    return [flat_rgb[3 * off[i]:3 * off[i + 1]].reshape(3, c.height, c.width)
            for i, c in enumerate(cams)]


def join_views(views):
    return np.concatenate([np.asarray(v, dtype=np.float64).ravel() for v in views])


# ------------------------------------------------------------------ entry points

def sh_basis(dirs: np.ndarray, deg: int) -> np.ndarray:
    dirs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((dirs.shape[0], (deg + 1) ** 2), dtype=np.float64)
    lib().ref_sh_basis(dirs.shape[0], deg, _p(dirs), _p(out))
    return out


def render(scene, cams, bg=(0.0, 0.0, 0.0), pix_list=None, wmax_in=None, threads=0):
    """FP64 forward (eq. 1-5).  Returns dict with flat rgb [3P] (view blocks),
    views (list of [3,H,W]), depth [P], alpha [P], n_hits [P], wmax [N]."""
    S = _SceneArrays(scene)
    c, wh = cams_arrays(cams)
    off = pix_offsets(cams)
    P = int(off[-1])
    rgb = np.zeros(3 * P, dtype=np.float64)
    depth = np.zeros(P, dtype=np.float64)
    alpha = np.zeros(P, dtype=np.float64)
    nh = np.zeros(P, dtype=np.int32)
    wmax = np.zeros(S.n, dtype=np.float64) if wmax_in is None else \
        np.ascontiguousarray(wmax_in, dtype=np.float64).copy()
    bgv = np.ascontiguousarray(bg, dtype=np.float64)
    pl = None if pix_list is None else np.ascontiguousarray(pix_list, dtype=np.int64)
    lib().ref_render(*S.args(), len(cams), _p(c), _p(wh), _p(bgv), _p(pl),
                     0 if pl is None else pl.shape[0], _p(rgb), _p(depth), _p(alpha),
                     _p(nh), _p(wmax), int(threads))
    return dict(rgb=rgb, views=split_views(rgb, cams), depth=depth, alpha=alpha,
                n_hits=nh, wmax=wmax)


def backward(scene, cams, g_rgb, g_depth=None, g_alpha=None, bg=(0.0, 0.0, 0.0),
             pix_list=None, threads=0):
    """FP64 analytic gradient (adjoint of eq. 2-4) -> (d_density [8,N], d_sh [K,N])."""
    S = _SceneArrays(scene)
    c, wh = cams_arrays(cams)
    g_rgb = np.ascontiguousarray(g_rgb, dtype=np.float64).ravel()
    gd = None if g_depth is None else np.ascontiguousarray(g_depth, dtype=np.float64).ravel()
    ga = None if g_alpha is None else np.ascontiguousarray(g_alpha, dtype=np.float64).ravel()
    dd = np.zeros((8, S.n), dtype=np.float64)
    dsh = np.zeros((3 * (S.deg + 1) ** 2, S.n), dtype=np.float64)
    bgv = np.ascontiguousarray(bg, dtype=np.float64)
    pl = None if pix_list is None else np.ascontiguousarray(pix_list, dtype=np.int64)
    lib().ref_backward(*S.args(), len(cams), _p(c), _p(wh), _p(bgv), _p(pl),
                       0 if pl is None else pl.shape[0], _p(g_rgb), _p(gd), _p(ga),
                       _p(dd), _p(dsh), int(threads))
    return dd, dsh


def render_aux(scene, cams, bg=(0.0, 0.0, 0.0), wmax_in=None, threads=0):
    """FP64 forward with the auxiliary channels: render()'s outputs plus
    dist [P] (per-pixel distortion) and normal [3P] (rendered normal, rgb
    layout: view blocks [3, H, W]); see raster_ref.cpp for the readings."""
    S = _SceneArrays(scene)
    c, wh = cams_arrays(cams)
    off = pix_offsets(cams)
    P = int(off[-1])
    rgb = np.zeros(3 * P, dtype=np.float64)
    depth = np.zeros(P, dtype=np.float64)
    alpha = np.zeros(P, dtype=np.float64)
    dist = np.zeros(P, dtype=np.float64)
    normal = np.zeros(3 * P, dtype=np.float64)
    wmax = np.zeros(S.n, dtype=np.float64) if wmax_in is None else \
        np.ascontiguousarray(wmax_in, dtype=np.float64).copy()
    bgv = np.ascontiguousarray(bg, dtype=np.float64)
    lib().ref_render_aux(*S.args(), len(cams), _p(c), _p(wh), _p(bgv), _p(rgb), _p(depth),
                         _p(alpha), _p(dist), _p(normal), _p(wmax), int(threads))
    return dict(rgb=rgb, views=split_views(rgb, cams), depth=depth, alpha=alpha, dist=dist,
                normal=normal, wmax=wmax)


def median_depth(scene, cams, t_half=0.5, threads=0):
    """FP64 median depth [P]: chord midpoint of the first hit after which the
    transmittance is at most t_half (0 where none is); see raster_ref.cpp."""
    S = _SceneArrays(scene)
    c, wh = cams_arrays(cams)
    P = int(pix_offsets(cams)[-1])
    md = np.zeros(P, dtype=np.float64)
    lib().ref_median_depth(*S.args(), len(cams), _p(c), _p(wh), float(t_half), _p(md),
                           int(threads))
    return md


def backward_aux(scene, cams, g_rgb, g_depth=None, g_alpha=None, g_dist=None, g_normal=None,
                 bg=(0.0, 0.0, 0.0), threads=0):
    """FP64 analytic gradient with the auxiliary channels -> (d_density, d_sh)."""
    S = _SceneArrays(scene)
    c, wh = cams_arrays(cams)
    f = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64).ravel()
    g_rgb, gd, ga, gl, gn = f(g_rgb), f(g_depth), f(g_alpha), f(g_dist), f(g_normal)
    dd = np.zeros((8, S.n), dtype=np.float64)
    dsh = np.zeros((3 * (S.deg + 1) ** 2, S.n), dtype=np.float64)
    bgv = np.ascontiguousarray(bg, dtype=np.float64)
    lib().ref_backward_aux(*S.args(), len(cams), _p(c), _p(wh), _p(bgv), _p(g_rgb), _p(gd),
                           _p(ga), _p(gl), _p(gn), _p(dd), _p(dsh), int(threads))
    return dd, dsh


def trace_pixel(scene, cam, px, py, cap=4096):
    """Per-hit record of one pixel ray, front to back."""
    S = _SceneArrays(scene)
    c, wh = cams_arrays([cam])
    vid = np.zeros(cap, np.int64)
    arrs = [np.zeros(cap, np.float64) for _ in range(5)]
    k = lib().ref_trace_pixel(*S.args(), _p(c), _p(wh), int(px), int(py), cap, _p(vid),
                              *[_p(a) for a in arrs])
    k = min(k, cap)
    tin, tout, tau, w, Ta = [a[:k] for a in arrs]
    return dict(vid=vid[:k], tin=tin, tout=tout, tau=tau, w=w, T_after=Ta)


def voxel_colours(scene, cams):
    """Raw SH sums and clamped colours per (view, voxel): two [V, N, 3] arrays."""
    S = _SceneArrays(scene)
    c, wh = cams_arrays(cams)
    raw = np.zeros((len(cams), S.n, 3), np.float64)
    col = np.zeros((len(cams), S.n, 3), np.float64)
    lib().ref_voxel_colours(S.n, S.deg, _p(S.root_min), S.root_size, _p(S.ijk), _p(S.level),
                            _p(S.sh), len(cams), _p(c), _p(wh), _p(raw), _p(col))
    return raw, col


def footprint_pixels(scene, cams, vox):
    S = _SceneArrays(scene)
    c, wh = cams_arrays(cams)
    vox = np.ascontiguousarray(vox, dtype=np.int64)
    cap = 1 << 20
    while True:
        out = np.zeros(cap, np.int64)
        k = lib().ref_footprint_pixels(S.n, _p(S.root_min), S.root_size, _p(S.ijk),
                                       _p(S.level), len(cams), _p(c), _p(wh), _p(vox),
                                       vox.shape[0], _p(out), cap)
        if k <= cap:
            return np.unique(out[:k])
        cap = int(k)


def project_keys(scene, cams, z_near=1e-4):
    """Binary32 key path: per (view, voxel) visibility, pixel-centre rect
    (x0, x1, y0, y1) and 36-bit visibility code."""
    S = _SceneArrays(scene)
    c, wh = cams_arrays(cams)
    V = len(cams)
    vis = np.zeros((V, S.n), np.uint8)
    rect = np.zeros((V, S.n, 4), np.int32)
    code = np.zeros((V, S.n), np.uint64)
    lib().ref_project_keys(S.n, _p(S.root_min), np.float32(S.root_size), _p(S.ijk),
                           _p(S.level), V, _p(c), _p(wh), np.float32(z_near),
                           _p(vis), _p(rect), _p(code))
    return vis, rect, code


def tile_lists(cams, vis, rect, code, tile):
    """Expand records into (global tile, code, voxel) pairs and sort them by
    key = tile << 36 | code (ties by voxel id).  Returns (tile_start [T+1],
    ids [Q], keys [Q]) with tiles numbered view by view, row-major."""
    bases = [0]
    for c in cams:
        bases.append(bases[-1] + ((c.width + tile - 1) // tile) * ((c.height + tile - 1) // tile))
    gts, codes, ids = [], [], []
    for v, c in enumerate(cams):
        tx_n = (c.width + tile - 1) // tile
        idx = np.nonzero(vis[v])[0]
        r = rect[v, idx]
        tx0, tx1, ty0, ty1 = r[:, 0] // tile, r[:, 1] // tile, r[:, 2] // tile, r[:, 3] // tile
        nx, ny = tx1 - tx0 + 1, ty1 - ty0 + 1
        cnt = nx * ny
        rep = np.repeat(np.arange(idx.shape[0]), cnt)
        start = np.repeat(np.cumsum(cnt) - cnt, cnt)
        k = np.arange(rep.shape[0]) - start
        tx = tx0[rep] + k % nx[rep]
        ty = ty0[rep] + k // nx[rep]
        gts.append(bases[v] + ty * tx_n + tx)
        codes.append(code[v, idx][rep])
        ids.append(idx[rep])
    gt = np.concatenate(gts).astype(np.uint64)
    cd = np.concatenate(codes).astype(np.uint64)
    vid = np.concatenate(ids).astype(np.uint64)
    keys = (gt << np.uint64(36)) | cd
    order = np.lexsort((vid, keys))
    keys, vid, gt = keys[order], vid[order], gt[order]
    T = bases[-1]
    start = np.searchsorted(gt, np.arange(T + 1, dtype=np.uint64), side="left").astype(np.int64)
    return start, vid.astype(np.int64), keys
