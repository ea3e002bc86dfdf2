"""Seeded synthetic scenes, cameras and target images.

Workloads stand in for the paper's Mip-NeRF 360 / Tanks & Temples training
views (Sec. V), which are not available: sparse octree leaves on a spherical
shell (optionally with uniform clutter), trilinear corner densities and SH
colour coefficients, pinhole cameras looking at the origin, and smooth target
images with a few hard edges so the inverse-Sobel weight (Sec. IV-B, eq. 7)
has both flat and edge regions to act on.

Layouts (structure of arrays, the same layout the C-ABI takes):
  ijk      uint16 [3, N]     integer cell coordinates at the leaf's level
  level    uint8  [N]        octree level l; edge = root_size * 2**-l
  density  float32 [8, N]    corner densities, corner c = x + 2*y + 4*z bits
  sh       float32 [K, N]    K = 3*(deg+1)**2, row (i*3 + channel), i = l*l+l+m

Cameras use OpenCV axes (x right, y down, z forward): x_cam = R (x - o).
The horizontal field of view is 50 degrees: fx = fy = (W/2)/tan(25 deg),
cx = W/2, cy = H/2.

Nothing here evaluates the rasterizer; every number is a draw from a seeded
numpy PCG64 generator.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

L_MAX = 12
FOV_X_DEG = 50.0
CAM_RADIUS = 2.5


@dataclasses.dataclass
class Scene:
    root_min: np.ndarray          # float32 [3]
    root_size: float              # S, edge of the cubic root cell
    ijk: np.ndarray               # uint16 [3, N]
    level: np.ndarray             # uint8 [N]
    density: np.ndarray           # float32 [8, N]
    sh: np.ndarray                # float32 [3*(deg+1)^2, N]
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.level.shape[0])


@dataclasses.dataclass
class Camera:
    R: np.ndarray                 # float32 [3, 3], rows = right, down, forward
    o: np.ndarray                 # float32 [3], camera centre
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def npix(self) -> int:
        return self.width * self.height


def config_seed(name: str) -> int:
    order = ["grid4k", "shell200k", "shell200k_train", "ring1m", "hemi4m"]
    return 251102510 + 1 + order.index(name)


# ----------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------

def look_at(o: Sequence[float], width: int, height: int,
            target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)) -> Camera:
    o64 = np.asarray(o, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - o64
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, dtype=np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f]).astype(np.float32)
    foc = (width / 2.0) / math.tan(math.radians(FOV_X_DEG / 2.0))
    return Camera(R=R, o=o64.astype(np.float32), fx=float(np.float32(foc)),
                  fy=float(np.float32(foc)), cx=width / 2.0, cy=height / 2.0,
                  width=int(width), height=int(height))


def make_cameras_single(width: int, height: int) -> List[Camera]:
    # a generic direction so that no ray grazes a face of the axis-aligned grid
    o = CAM_RADIUS * np.array([0.48, 0.36, 0.80])
    return [look_at(o, width, height)]


RING_RESOLUTIONS = [(640, 480), (1024, 768), (1280, 720), (1600, 1080)]


def make_cameras_ring(rng: np.random.Generator, n_views: int = 8,
                      elevation_deg: float = 11.5) -> List[Camera]:
    el = math.radians(elevation_deg)
    cams = []
    picks = rng.integers(0, len(RING_RESOLUTIONS), size=n_views)
    for i in range(n_views):
        az = 2.0 * math.pi * i / n_views + 0.1
        o = CAM_RADIUS * np.array([math.cos(el) * math.cos(az), math.sin(el),
                                   math.cos(el) * math.sin(az)])
        w, h = RING_RESOLUTIONS[int(picks[i])]
        cams.append(look_at(o, w, h))
    return cams


def make_cameras_hemisphere(n_views: int = 16, width: int = 1920,
                            height: int = 1080) -> List[Camera]:
    golden = math.pi * (3.0 - math.sqrt(5.0))
    cams = []
    for i in range(n_views):
        y = 0.15 + 0.80 * (i + 0.5) / n_views
        rxz = math.sqrt(max(0.0, 1.0 - y * y))
        az = golden * i
        o = CAM_RADIUS * np.array([rxz * math.cos(az), y, rxz * math.sin(az)])
        cams.append(look_at(o, width, height))
    return cams


# ----------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------

def _softplus(x: np.ndarray) -> np.ndarray:
    return np.logaddexp(0.0, x)


def _draw_params(rng: np.random.Generator, n: int, density_std: float,
                 sh_degree: int):
    density = _softplus(rng.normal(0.0, density_std, size=(8, n))).astype(np.float32)
    k = 3 * (sh_degree + 1) ** 2
    sh = np.empty((k, n), dtype=np.float32)
    sh[0:3] = rng.uniform(0.0, 1.0, size=(3, n))
    if k > 3:
        sh[3:] = rng.normal(0.0, 0.1, size=(k - 3, n))
    return density, sh


def make_scene_grid(rng: np.random.Generator, res_level: int = 4,
                    sh_degree: int = 0, density_std: float = 1.0) -> Scene:
    """Uniform grid of 2**res_level cells per axis filling the root cube
    [-0.5, 0.5]^3 (one octree level)."""
    g = 1 << res_level
    iz, iy, ix = np.meshgrid(np.arange(g), np.arange(g), np.arange(g), indexing="ij")
    ijk = np.stack([ix.ravel(), iy.ravel(), iz.ravel()]).astype(np.uint16)
    n = ijk.shape[1]
    level = np.full(n, res_level, dtype=np.uint8)
    order = octree_order(ijk, level)
    ijk = np.ascontiguousarray(ijk[:, order])
    density, sh = _draw_params(rng, n, density_std, sh_degree)
    return Scene(root_min=np.array([-0.5, -0.5, -0.5], np.float32), root_size=1.0,
                 ijk=ijk, level=level, density=density, sh=sh, sh_degree=sh_degree)


def octree_order(ijk: np.ndarray, level: np.ndarray) -> np.ndarray:
    """Permutation that puts leaves in octree depth-first order.

    A sparse voxel octree stores its leaves in this order (the order of a
    depth-first walk, children in z, y, x bit order); it is the storage
    order of every generated scene.  Key: the bits of the leaf's minimum
    corner at the finest level, interleaved (x lowest)."""
    c = [ijk[a].astype(np.int64) << (L_MAX - level.astype(np.int64)) for a in range(3)]
    key = np.zeros(ijk.shape[1], dtype=np.int64)
    for b in range(L_MAX):
        for a in range(3):
            key |= ((c[a] >> b) & 1) << (3 * b + a)
    return np.argsort(key, kind="stable")


def _key(ix, iy, iz):
    return ix.astype(np.int64) | (iy.astype(np.int64) << 12) | (iz.astype(np.int64) << 24)


def _level_counts(n: int, lmin: int, lmax: int) -> np.ndarray:
    lv = np.arange(lmin, lmax + 1)
    p = np.exp2(lv.astype(np.float64))
    p /= p.sum()
    raw = n * p
    cnt = np.floor(raw).astype(np.int64)
    rem = n - int(cnt.sum())
    order = np.argsort(-(raw - cnt), kind="stable")
    cnt[order[:rem]] += 1
    return cnt


def _shell_points(rng, m, r_lo, r_hi):
    v = rng.normal(size=(m, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = rng.uniform(r_lo, r_hi, size=(m, 1))
    return v * r


def make_scene_shell(rng: np.random.Generator, n: int, lmin: int, lmax: int,
                     sh_degree: int = 3, density_std: float = 2.0,
                     clutter_frac: float = 0.0, r_lo: float = 0.75,
                     r_hi: float = 0.85) -> Scene:
    """Sparse octree leaves in the root cube [-1, 1]^3.

    Leaf levels follow P(l) proportional to 2**l on [lmin, lmax]; a leaf is the
    cell containing a point drawn on the shell r in [r_lo, r_hi] (uniform
    direction), or, for a clutter_frac share, uniformly in the root cube.
    Levels are filled coarse to fine; a candidate cell is rejected when it
    duplicates an accepted leaf or lies inside a coarser accepted leaf, so the
    leaves never overlap.  The leaves are returned in octree order.
    """
    assert 0 <= lmin <= lmax <= L_MAX
    root_min = np.array([-1.0, -1.0, -1.0], np.float32)
    S = 2.0
    counts = _level_counts(n, lmin, lmax)
    accepted = {}          # level -> sorted int64 keys
    out_ijk, out_lv = [], []
    for li, l in enumerate(range(lmin, lmax + 1)):
        need_total = int(counts[li])
        need_clutter = int(round(clutter_frac * need_total))
        quotas = [(need_total - need_clutter, False), (need_clutter, True)]
        e = S / (1 << l)
        got_level = np.zeros(0, dtype=np.int64)
        for need, clutter in quotas:
            got = []
            n_got = 0
            rounds = 0
            while n_got < need:
                rounds += 1
                if rounds > 200:
                    raise ValueError(f"cannot place {need} leaves at level {l}: "
                                     "too few free cells for this level range")
                m = max(2 * (need - n_got) + 256, 1024)
                if clutter:
                    pts = rng.uniform(-1.0, 1.0, size=(m, 3))
                else:
                    pts = _shell_points(rng, m, r_lo, r_hi)
                idx = np.floor((pts - root_min.astype(np.float64)) / e).astype(np.int64)
                idx = np.clip(idx, 0, (1 << l) - 1)
                keys = _key(idx[:, 0], idx[:, 1], idx[:, 2])
                _, first = np.unique(keys, return_index=True)
                first.sort()
                idx, keys = idx[first], keys[first]
                ok = ~np.isin(keys, got_level)
                for lc, ak in accepted.items():
                    sh_ = l - lc
                    anc = _key(idx[:, 0] >> sh_, idx[:, 1] >> sh_, idx[:, 2] >> sh_)
                    ok &= ~np.isin(anc, ak)
                idx, keys = idx[ok], keys[ok]
                take = min(need - n_got, idx.shape[0])
                got.append(idx[:take])
                got_level = np.union1d(got_level, keys[:take])
                n_got += take
            if got:
                g = np.concatenate(got, axis=0)
                out_ijk.append(g)
                out_lv.append(np.full(g.shape[0], l, dtype=np.uint8))
        accepted[l] = got_level
    ijk = np.concatenate(out_ijk, axis=0).T.astype(np.uint16)
    level = np.concatenate(out_lv)
    rng.permutation(level.shape[0])   # keeps the later draws of each seed unchanged
    perm = octree_order(ijk, level)
    ijk = np.ascontiguousarray(ijk[:, perm])
    level = np.ascontiguousarray(level[perm])
    density, sh = _draw_params(rng, level.shape[0], density_std, sh_degree)
    return Scene(root_min=root_min, root_size=S, ijk=ijk, level=level,
                 density=density, sh=sh, sh_degree=sh_degree)


def scene_subset(scene: Scene, idx) -> Scene:
    idx = np.asarray(idx)
    return Scene(root_min=scene.root_min.copy(), root_size=scene.root_size,
                 ijk=np.ascontiguousarray(scene.ijk[:, idx]),
                 level=np.ascontiguousarray(scene.level[idx]),
                 density=np.ascontiguousarray(scene.density[:, idx]),
                 sh=np.ascontiguousarray(scene.sh[:, idx]), sh_degree=scene.sh_degree)


# ----------------------------------------------------------------------------
# target images
# ----------------------------------------------------------------------------

def grid_points(scene: Scene):
    """Shared corner points of a leaf set (grid-point storage): corner c of
    leaf v (c = x + 2y + 4z bits) lies at the finest-level coordinate
    (ijk + bits) * 2^(L_MAX - l); leaves whose corners coincide share one
    point (a corner in the middle of a coarser leaf's face or edge is a point
    of its own).  Returns (corner_idx int32 [8][N], n_grid), points numbered
    in the order of their first appearance."""
    n = scene.n
    shift = (L_MAX - scene.level.astype(np.int64))
    keys = np.empty((8, n), dtype=np.int64)
    for c in range(8):
        x = (scene.ijk[0].astype(np.int64) + (c & 1)) << shift
        y = (scene.ijk[1].astype(np.int64) + ((c >> 1) & 1)) << shift
        z = (scene.ijk[2].astype(np.int64) + ((c >> 2) & 1)) << shift
        keys[c] = x | (y << 13) | (z << 26)
    flat = keys.T.ravel()                       # voxel-major: first appearance order
    uniq, first, inv = np.unique(flat, return_index=True, return_inverse=True)
    rank = np.empty(uniq.shape[0], dtype=np.int64)
    rank[np.argsort(first, kind="stable")] = np.arange(uniq.shape[0])
    idx = rank[inv].reshape(n, 8).T
    return np.ascontiguousarray(idx, dtype=np.int32), int(uniq.shape[0])


def make_target(rng: np.random.Generator, width: int, height: int) -> np.ndarray:
    """float32 [3, H, W]: 0.5 + six low-frequency sinusoids (at most 4 cycles
    per image, amplitude 0.08) + three half-plane steps (amplitude 0.25) per
    channel, clipped to [0, 1]."""
    y, x = np.meshgrid((np.arange(height) + 0.5) / height,
                       (np.arange(width) + 0.5) / width, indexing="ij")
    img = np.empty((3, height, width), dtype=np.float64)
    for ch in range(3):
        acc = np.full((height, width), 0.5)
        for _ in range(6):
            fx, fy = rng.uniform(-4.0, 4.0, size=2)
            ph = rng.uniform(0.0, 2.0 * math.pi)
            acc += 0.08 * np.sin(2.0 * math.pi * (fx * x + fy * y) + ph)
        for _ in range(3):
            th = rng.uniform(0.0, 2.0 * math.pi)
            px, py = rng.uniform(0.2, 0.8, size=2)
            side = (x - px) * math.cos(th) + (y - py) * math.sin(th) > 0.0
            acc += np.where(side, 0.25, 0.0) * (1.0 if rng.uniform() < 0.5 else -1.0)
        img[ch] = acc
    return np.clip(img, 0.0, 1.0).astype(np.float32)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

CONFIGS = {
    # 4,096 voxels on a 16^3 grid, SH0, one 64x64 view, L1 x inverse-Sobel (gamma 0.5)
    "grid4k": dict(kind="grid", sh_degree=0),
    # 200k voxels levels 6-10 on a shell, SH3, one 800x600 view, forward + w_max
    "shell200k": dict(kind="shell", n=200_000, lmin=6, lmax=10, views="single",
                      width=800, height=600),
    # same scene, fwd+bwd with the inverse-Sobel L1 loss
    "shell200k_train": dict(kind="shell", n=200_000, lmin=6, lmax=10, views="single",
                            width=800, height=600, same_as="shell200k"),
    # 1M voxels levels 7-11, 10% clutter, 8 ring views of uneven resolution
    "ring1m": dict(kind="shell", n=1_000_000, lmin=7, lmax=11, clutter=0.1, views="ring"),
    # 4M voxels levels 8-12, 16 views 1920x1080 on a hemisphere
    "hemi4m": dict(kind="shell", n=4_000_000, lmin=8, lmax=12, views="hemi"),
}


def make_config(name: str, n_override: Optional[int] = None):
    """Return (scene, cameras, targets) for a named workload."""
    spec = CONFIGS[name]
    seed_name = spec.get("same_as", name)
    rng = np.random.default_rng(config_seed(seed_name))
    if spec["kind"] == "grid":
        scene = make_scene_grid(rng, 4, sh_degree=spec["sh_degree"], density_std=1.0)
        cams = make_cameras_single(64, 64)
    else:
        n = n_override if n_override is not None else spec["n"]
        scene = make_scene_shell(rng, n, spec["lmin"], spec["lmax"], sh_degree=3,
                                 density_std=2.0, clutter_frac=spec.get("clutter", 0.0))
        if spec["views"] == "single":
            cams = make_cameras_single(spec["width"], spec["height"])
        elif spec["views"] == "ring":
            cams = make_cameras_ring(rng, 8)
        else:
            cams = make_cameras_hemisphere(16, 1920, 1080)
    trng = np.random.default_rng(config_seed(seed_name) + 1000)
    targets = [make_target(trng, c.width, c.height) for c in cams]
    return scene, cams, targets
