"""Thin Python binding of liblitevoxel (argument marshalling only).

Device memory and streams come from PyTorch; every step of the rasterizer runs
in the library's HIP kernels.  Function names follow the C-ABI
(lv_forward -> forward, ...).  The only host logic here is bookkeeping: the
pair-capacity re-plan after lv_check_overflow and the torch.autograd.Function
that pairs lv_forward with lv_backward.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _abi
from ._abi import LvCamera, LvFrame, LvSettings, LvVoxels


class LiteVoxelError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    """An lv_context bound to one HIP device."""

    def __init__(self, device: int = 0):
        self.lib = _abi.lib()
        h = ctypes.c_void_p()
        s = self.lib.lv_create(ctypes.byref(h), int(device))
        if s != _abi.LV_OK:
            raise LiteVoxelError(s, f"lv_create(device={device}): "
                                 f"{self.lib.lv_status_str(s).decode()}")
        self.h = h
        self.device = torch.device("cuda", int(device))

    def check(self, s: int, what: str):
        if s != _abi.LV_OK:
            msg = self.lib.lv_last_error(self.h).decode()
            raise LiteVoxelError(s, f"{what}: {self.lib.lv_status_str(s).decode()}: {msg}")

    def close(self):
        if getattr(self, "h", None):
            self.lib.lv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Voxels:
    """Voxel leaves in device memory (structure of arrays).  Dense layout:
    density [8, n], one value per corner.  Grid-point layout: density
    [n_grid] on shared corner points and corner_idx [8, n] (int32); act is
    the density activation (_abi.ACT_*) applied to every stored value."""

    def __init__(self, ijk: torch.Tensor, level: torch.Tensor, density: torch.Tensor,
                 sh: torch.Tensor, root_min, root_size: float, sh_degree: int,
                 corner_idx: Optional[torch.Tensor] = None, act: int = 0):
        self.ijk, self.level, self.density, self.sh = ijk, level, density, sh
        self.corner_idx = corner_idx
        self.act = int(act)
        self.root_min = [float(x) for x in root_min]
        self.root_size = float(root_size)
        self.sh_degree = int(sh_degree)
        self.n = int(level.shape[0])
        self.n_grid = int(density.shape[0]) if corner_idx is not None else 0
        self.struct = self._make(density, sh)

    def _make(self, density, sh) -> LvVoxels:
        s = LvVoxels()
        s.n = self.n
        s.sh_degree = self.sh_degree
        s.root_min = (ctypes.c_float * 3)(*self.root_min)
        s.root_size = self.root_size
        s.ijk = self.ijk.data_ptr() if self.n else None
        s.level = self.level.data_ptr() if self.n else None
        s.density = density.data_ptr() if density.numel() else None
        s.sh = sh.data_ptr() if self.n else None
        s.corner_idx = self.corner_idx.data_ptr() if (self.corner_idx is not None and self.n) else None
        s.n_grid = self.n_grid
        s.density_act = self.act
        return s

    def with_params(self, density: torch.Tensor, sh: torch.Tensor) -> "Voxels":
        v = Voxels.__new__(Voxels)
        v.__dict__.update(self.__dict__)
        v.density, v.sh = density, sh
        v.struct = v._make(density, sh)
        return v

    @staticmethod
    def from_grid(scene, corner_idx, grid_values, device, act: int = 0) -> "Voxels":
        """The leaves of `scene` with grid-point densities: corner_idx [8, n],
        grid_values [n_grid] (the scene's own density rows are not used)."""
        dev = torch.device(device)
        ijk = torch.from_numpy(np.ascontiguousarray(scene.ijk).view(np.int16)).to(dev)
        level = torch.from_numpy(np.ascontiguousarray(scene.level)).to(dev)
        idx = torch.from_numpy(np.ascontiguousarray(corner_idx, dtype=np.int32)).to(dev)
        vals = torch.from_numpy(np.ascontiguousarray(grid_values, dtype=np.float32)).to(dev)
        sh = torch.from_numpy(np.ascontiguousarray(scene.sh, dtype=np.float32)).to(dev)
        return Voxels(ijk, level, vals, sh, scene.root_min, scene.root_size, scene.sh_degree,
                      corner_idx=idx, act=act)

    @staticmethod
    def from_scene(scene, device, act: int = 0) -> "Voxels":
        dev = torch.device(device)
        ijk = torch.from_numpy(np.ascontiguousarray(scene.ijk).view(np.int16)).to(dev)
        level = torch.from_numpy(np.ascontiguousarray(scene.level)).to(dev)
        dens = torch.from_numpy(np.ascontiguousarray(scene.density, dtype=np.float32)).to(dev)
        sh = torch.from_numpy(np.ascontiguousarray(scene.sh, dtype=np.float32)).to(dev)
        return Voxels(ijk, level, dens, sh, scene.root_min, scene.root_size, scene.sh_degree, act=act)


class Frame:
    """A batch of pinhole views (host copy for planning, device copy for kernels)."""

    def __init__(self, cams: Sequence, device, bg=(0.0, 0.0, 0.0)):
        self.n_views = len(cams)
        self.host = (LvCamera * self.n_views)()
        for i, c in enumerate(cams):
            self._fill(self.host[i], c)
        raw = np.frombuffer(bytes(self.host), dtype=np.uint8).copy()
        self.dev = torch.from_numpy(raw).to(torch.device(device))
        self.sizes = [(int(c.width), int(c.height)) for c in cams]
        self.off = np.zeros(self.n_views + 1, dtype=np.int64)
        for i, (w, h) in enumerate(self.sizes):
            self.off[i + 1] = self.off[i] + w * h
        self.P = int(self.off[-1])
        self.struct = LvFrame()
        self.struct.n_views = self.n_views
        self.struct.cams_host = ctypes.cast(self.host, ctypes.POINTER(LvCamera))
        self.struct.cams_dev = self.dev.data_ptr()
        self.struct.bg = (ctypes.c_float * 3)(*[float(x) for x in bg])

    @staticmethod
    def _fill(dst: LvCamera, c):
        R = np.asarray(c.R, dtype=np.float32).ravel()
        dst.R = (ctypes.c_float * 9)(*R.tolist())
        dst.o = (ctypes.c_float * 3)(*np.asarray(c.o, dtype=np.float32).tolist())
        dst.fx, dst.fy, dst.cx, dst.cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        dst.width, dst.height = int(c.width), int(c.height)

    def set_poses(self, cams: Sequence):
        """Replace the cameras in place (same sizes): graph replays read the new poses."""
        assert len(cams) == self.n_views
        for i, c in enumerate(cams):
            assert (int(c.width), int(c.height)) == self.sizes[i], "sizes are fixed"
            self._fill(self.host[i], c)
        raw = torch.from_numpy(np.frombuffer(bytes(self.host), dtype=np.uint8).copy())
        self.dev.copy_(raw, non_blocking=False)

    def view_rgb(self, rgb: torch.Tensor, v: int) -> torch.Tensor:
        w, h = self.sizes[v]
        return rgb[3 * self.off[v]:3 * self.off[v + 1]].view(3, h, w)


def settings(tile=16, chunk=64, t_eps=1e-6, pair_capacity=0, chunk_bwd=0) -> LvSettings:
    """chunk: voxels staged per step of the forward; chunk_bwd: of the
    backward (0: the same as chunk)."""
    s = LvSettings()
    s.tile, s.chunk, s.chunk_bwd = int(tile), int(chunk), int(chunk_bwd)
    s.t_eps, s.pair_capacity = float(t_eps), int(pair_capacity)
    return s


# --------------------------------------------------------------- C-ABI calls

def query_sizes(ctx: Context, vox: Voxels, frame: Frame, st: LvSettings):
    """-> (workspace_bytes, saved_bytes)."""
    ws, sv = ctypes.c_uint64(), ctypes.c_uint64()
    ctx.check(ctx.lib.lv_query_sizes(ctx.h, ctypes.byref(vox.struct), ctypes.byref(frame.struct),
                                     ctypes.byref(st), ctypes.byref(ws), ctypes.byref(sv)),
              "lv_query_sizes")
    return int(ws.value), int(sv.value)


def forward(ctx, vox, frame, st, workspace, saved, rgb, depth, alpha, wmax, stream=None):
    ctx.check(ctx.lib.lv_forward(ctx.h, ctypes.byref(vox.struct), ctypes.byref(frame.struct),
                                 ctypes.byref(st), _p(workspace), _p(saved), _p(rgb), _p(depth),
                                 _p(alpha), _p(wmax), _stream(stream)), "lv_forward")


def backward(ctx, vox, frame, st, workspace, saved, d_rgb, d_depth, d_alpha, d_density, d_sh,
             stream=None):
    ctx.check(ctx.lib.lv_backward(ctx.h, ctypes.byref(vox.struct), ctypes.byref(frame.struct),
                                  ctypes.byref(st), _p(workspace), _p(saved), _p(d_rgb),
                                  _p(d_depth), _p(d_alpha), _p(d_density), _p(d_sh),
                                  _stream(stream)), "lv_backward")


def forward_aux(ctx, vox, frame, st, workspace, saved, rgb, depth, alpha, wmax, dist, normal,
                mdepth=None, stream=None):
    """lv_forward_aux: lv_forward plus the distortion [P], normal [3P] and
    median-depth [P] channels (each may be None)."""
    ctx.check(ctx.lib.lv_forward_aux(ctx.h, ctypes.byref(vox.struct), ctypes.byref(frame.struct),
                                     ctypes.byref(st), _p(workspace), _p(saved), _p(rgb),
                                     _p(depth), _p(alpha), _p(wmax), _p(dist), _p(normal),
                                     _p(mdepth), _stream(stream)), "lv_forward_aux")


def backward_aux(ctx, vox, frame, st, workspace, saved, d_rgb, d_depth, d_alpha, depth_fwd,
                 d_dist, d_normal, d_density, d_sh, stream=None):
    ctx.check(ctx.lib.lv_backward_aux(ctx.h, ctypes.byref(vox.struct), ctypes.byref(frame.struct),
                                      ctypes.byref(st), _p(workspace), _p(saved), _p(d_rgb),
                                      _p(d_depth), _p(d_alpha), _p(depth_fwd), _p(d_dist),
                                      _p(d_normal), _p(d_density), _p(d_sh), _stream(stream)),
              "lv_backward_aux")


def aux_loss(ctx, frame, depth, alpha, normal, dist, lam_tc, lam_n, lam_d, loss, d_alpha,
             d_depth, d_normal, d_dist, stream=None, mdepth=None, lam_nm=0.0):
    """lv_aux_loss: per-view transmittance-concentration, depth-normal,
    distortion and (with mdepth) median depth-normal terms (loss [4 V]) and
    their gradients."""
    ctx.check(ctx.lib.lv_aux_loss(ctx.h, ctypes.byref(frame.struct), _p(depth), _p(alpha),
                                  _p(normal), _p(dist), _p(mdepth), float(lam_tc), float(lam_n),
                                  float(lam_d), float(lam_nm), _p(loss), _p(d_alpha), _p(d_depth),
                                  _p(d_normal), _p(d_dist), _stream(stream)), "lv_aux_loss")


def check_overflow(ctx, vox, frame, st, saved, stream=None):
    """(fits, pairs_needed) of the forward pass that filled `saved`;
    synchronises the stream."""
    need = ctypes.c_uint64()
    s = ctx.lib.lv_check_overflow(ctx.h, ctypes.byref(vox.struct), ctypes.byref(frame.struct),
                                  ctypes.byref(st), _p(saved), ctypes.byref(need),
                                  _stream(stream))
    if s == _abi.LV_ERR_CAPACITY:
        return False, int(need.value)
    ctx.check(s, "lv_check_overflow")
    return True, int(need.value)


def pass_stats(ctx, vox, frame, st, saved, stream=None):
    """(pairs, visible records) of the forward pass that filled `saved`;
    synchronises the stream."""
    q, m = ctypes.c_uint64(), ctypes.c_uint64()
    ctx.check(ctx.lib.lv_pass_stats(ctx.h, ctypes.byref(vox.struct), ctypes.byref(frame.struct),
                                    ctypes.byref(st), _p(saved), ctypes.byref(q), ctypes.byref(m),
                                    _stream(stream)), "lv_pass_stats")
    return int(q.value), int(m.value)


def export_bins(ctx, vox, frame, st, saved, stream=None):
    """Host copies of the binning state a forward pass left in `saved`:
    dict(tile_start, ids, codes, rects, vis)."""
    T = 0
    for (w, h) in frame.sizes:
        T += ((w + st.tile - 1) // st.tile) * ((h + st.tile - 1) // st.tile)
    ts = np.zeros(T + 1, dtype=np.uint32)
    nr = vox.n * frame.n_views
    codes = np.zeros(nr, dtype=np.uint64)
    rects = np.zeros((nr, 4), dtype=np.int32)
    vis = np.zeros(nr, dtype=np.uint8)
    cap = int(st.pair_capacity)
    ids = np.zeros(max(cap, 1), dtype=np.uint32)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    ctx.check(ctx.lib.lv_export_bins(ctx.h, ctypes.byref(vox.struct), ctypes.byref(frame.struct),
                                     ctypes.byref(st), _p(saved), ptr(ts), ptr(ids), ptr(codes),
                                     ptr(rects), ptr(vis), _stream(stream)), "lv_export_bins")
    tot = min(int(ts[-1]), cap)
    return dict(tile_start=ts.astype(np.int64), ids=ids[:tot].astype(np.int64),
                codes=codes.reshape(frame.n_views, vox.n), rects=rects.reshape(frame.n_views, vox.n, 4),
                vis=vis.reshape(frame.n_views, vox.n))


def lf_weight_workspace_size(n_views: int) -> int:
    return int(_abi.lib().lv_lf_weight_workspace_size(int(n_views)))


def lf_weight(ctx, frame, target, gamma, form, eps, weight, workspace, stream=None):
    ctx.check(ctx.lib.lv_lf_weight(ctx.h, ctypes.byref(frame.struct), _p(target), float(gamma),
                                   int(form), float(eps), _p(weight), _p(workspace),
                                   _stream(stream)), "lv_lf_weight")


def lf_weight_noalloc(ctx, frame, target, gamma, form, eps, weight, stream=None):
    """lf_weight on the library's static scratch (no workspace argument; at
    most 64 views; calls overlapping on one GPU race)."""
    ctx.check(ctx.lib.lv_lf_weight_noalloc(ctx.h, ctypes.byref(frame.struct), _p(target),
                                           float(gamma), int(form), float(eps), _p(weight),
                                           _stream(stream)), "lv_lf_weight_noalloc")


def l1_grad(ctx, frame, rgb, target, weight, loss, d_rgb, stream=None):
    ctx.check(ctx.lib.lv_l1_grad(ctx.h, ctypes.byref(frame.struct), _p(rgb), _p(target),
                                 _p(weight), _p(loss), _p(d_rgb), _stream(stream)), "lv_l1_grad")


def gamma_schedule(t, total, t0_frac=0.3, t1_frac=0.6, gamma_max=0.6) -> float:
    return float(_abi.lib().lv_gamma_schedule(float(t), float(total), float(t0_frac),
                                              float(t1_frac), float(gamma_max)))


def quantile_workspace_size(n: int, n_bins: int) -> int:
    return int(_abi.lib().lv_quantile_workspace_size(int(n), int(n_bins)))


def depth_quantile(ctx, vox, frame, wmax, n_bins, q, workspace, tau, prune, bins=None, stream=None):
    ctx.check(ctx.lib.lv_depth_quantile(ctx.h, ctypes.byref(vox.struct), ctypes.byref(frame.struct),
                                        _p(wmax), int(n_bins), float(q), _p(workspace), _p(tau),
                                        _p(prune), _p(bins), _stream(stream)), "lv_depth_quantile")


def depth_bins(ctx, vox, frame, n_bins, workspace, bins=None, stream=None):
    """The w_max-independent half of depth_quantile (delta, p5/p95, bins) into
    workspace; depth_cutoff finishes it once w_max is known."""
    ctx.check(ctx.lib.lv_depth_bins(ctx.h, ctypes.byref(vox.struct), ctypes.byref(frame.struct),
                                    int(n_bins), _p(workspace), _p(bins), _stream(stream)),
              "lv_depth_bins")


def depth_cutoff(ctx, vox, wmax, n_bins, q, workspace, tau, prune, stream=None):
    """tau and prune from w_max on a workspace filled by depth_bins."""
    ctx.check(ctx.lib.lv_depth_cutoff(ctx.h, ctypes.byref(vox.struct), _p(wmax), int(n_bins),
                                      float(q), _p(workspace), _p(tau), _p(prune), _stream(stream)),
              "lv_depth_cutoff")


def guard_params(**kw):
    """lv_guard_params with the library defaults, overridden by keyword
    (alpha, m_low, m_high, rho, w_keep, cap_frac)."""
    p = _abi.LvGuardParams()
    _abi.lib().lv_default_guard(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown guard parameter {k}")
        setattr(p, k, v)
    return p


def guard_workspace_size(n: int) -> int:
    return int(_abi.lib().lv_guard_workspace_size(int(n)))


def prune_guard(ctx, vox, frame, wmax, bins, tau, n_bins, params, workspace, ema, state, prune,
                n_pruned=None, stream=None):
    """One adaptation step of the pruning guards (lv_prune_guard): updates
    ema and state in place and writes prune."""
    ctx.check(ctx.lib.lv_prune_guard(ctx.h, ctypes.byref(vox.struct), ctypes.byref(frame.struct),
                                     _p(wmax), _p(bins), _p(tau), int(n_bins), ctypes.byref(params),
                                     _p(workspace), _p(ema), _p(state), _p(prune), _p(n_pruned),
                                     _stream(stream)), "lv_prune_guard")


def split_params(**kw):
    """lv_split_params with the library defaults (kappa 1, beta 0.2,
    max_splits 8192), overridden by keyword."""
    p = _abi.LvSplitParams()
    _abi.lib().lv_default_split(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown split parameter {k}")
        setattr(p, k, v)
    return p


def split_workspace_size(n: int) -> int:
    return int(_abi.lib().lv_split_workspace_size(int(n)))


def footprint_range(ctx, vox, frame, workspace, range_out, stream=None):
    """range_out [2] (device f32) = 5th and 95th percentiles of the footprint."""
    ctx.check(ctx.lib.lv_footprint_range(ctx.h, ctypes.byref(vox.struct), ctypes.byref(frame.struct),
                                         _p(workspace), _p(range_out), _stream(stream)),
              "lv_footprint_range")


def subdivide_select(ctx, vox, frame, score, range_in, params, workspace, split, priority=None,
                     n_split=None, stream=None):
    ctx.check(ctx.lib.lv_subdivide_select(ctx.h, ctypes.byref(vox.struct), ctypes.byref(frame.struct),
                                          _p(score), _p(range_in), ctypes.byref(params),
                                          _p(workspace), _p(split), _p(priority), _p(n_split),
                                          _stream(stream)), "lv_subdivide_select")


def subdivide_apply(ctx, vox, split, n_out, workspace, n_needed=None, stream=None) -> "Voxels":
    """The refined voxel set with n_out = n + 7 (#split) leaves (new device
    arrays; vox is left as it is)."""
    dev = vox.level.device
    n_out = int(n_out)
    K = 3 * (vox.sh_degree + 1) ** 2
    ijk = torch.empty((3, n_out), dtype=torch.int16, device=dev)
    level = torch.empty(n_out, dtype=torch.uint8, device=dev)
    dens = torch.empty((8, n_out), dtype=torch.float32, device=dev)
    sh = torch.empty((K, n_out), dtype=torch.float32, device=dev)
    ctx.check(ctx.lib.lv_subdivide_apply(ctx.h, ctypes.byref(vox.struct), _p(split), n_out,
                                         _p(workspace), _p(ijk), _p(level), _p(dens), _p(sh),
                                         _p(n_needed), _stream(stream)), "lv_subdivide_apply")
    return Voxels(ijk, level, dens, sh, vox.root_min, vox.root_size, vox.sh_degree, act=vox.act)


def graph_begin(ctx, stream):
    ctx.check(ctx.lib.lv_graph_begin(ctx.h, _stream(stream)), "lv_graph_begin")


def graph_end(ctx, stream):
    ctx.check(ctx.lib.lv_graph_end(ctx.h, _stream(stream)), "lv_graph_end")


def graph_launch(ctx, stream=None):
    ctx.check(ctx.lib.lv_graph_launch(ctx.h, _stream(stream)), "lv_graph_launch")


def graph_reset(ctx):
    ctx.check(ctx.lib.lv_graph_reset(ctx.h), "lv_graph_reset")


def tune_key(vox, frame) -> str:
    """Workload class an autotuning result is reused for: voxel count rounded
    to a power of two, view count, the multiset of resolutions, SH degree."""
    n = int(vox.n)
    bucket = n.bit_length() if n > 0 else 0
    res = ",".join(f"{w}x{h}" for w, h in sorted(frame.sizes))
    return f"n2^{bucket}|v{frame.n_views}|{res}|sh{int(vox.sh_degree)}"


def autotune(ctx, vox, frame, reps=3, t_eps=1e-6, stream=None, cache=None):
    """-> (best LvSettings, ms table [forward, backward] x 3 tiles x 3 chunks).

    The best setting takes the tile whose fastest forward plus fastest
    backward is smallest, and those two chunks as chunk and chunk_bwd.
    cache: optional path of a JSON file of earlier results keyed by tune_key;
    a hit returns the stored tile and chunks (pair capacity 0: the Renderer
    plans it) without timing anything, a miss times and stores."""
    import json
    import os
    key = tune_key(vox, frame)
    if cache is not None and os.path.exists(cache):
        with open(cache) as fh:
            known = json.load(fh)
        hit = known.get(key)
        if hit is not None and "chunk_bwd" in hit and len(hit["ms_table"]) == 18:
            return (settings(tile=int(hit["tile"]), chunk=int(hit["chunk"]), t_eps=t_eps,
                             chunk_bwd=int(hit["chunk_bwd"])),
                    np.array(hit["ms_table"], dtype=np.float64).reshape(2, 3, 3))
    best = settings(t_eps=t_eps)
    table = (ctypes.c_float * 18)()
    ctx.check(ctx.lib.lv_autotune(ctx.h, ctypes.byref(vox.struct), ctypes.byref(frame.struct),
                                  int(reps), ctypes.byref(best), ctypes.cast(table, ctypes.c_void_p),
                                  _stream(stream)), "lv_autotune")
    ms = np.array(list(table), dtype=np.float64).reshape(2, 3, 3)
    if cache is not None:
        known = {}
        if os.path.exists(cache):
            with open(cache) as fh:
                known = json.load(fh)
        known[key] = {"tile": int(best.tile), "chunk": int(best.chunk),
                      "chunk_bwd": int(best.chunk_bwd),
                      "ms_table": [round(float(x), 4) for x in ms.ravel()]}
        tmp = f"{cache}.tmp{os.getpid()}"
        with open(tmp, "w") as fh:
            json.dump(known, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return best, ms


def set_timing(ctx, enable: bool):
    ctx.check(ctx.lib.lv_set_timing(ctx.h, 1 if enable else 0), "lv_set_timing")


def read_timings(ctx):
    """Synchronises; per-phase (ms, launches) since the last read."""
    ms = (ctypes.c_double * len(_abi.PHASES))()
    calls = (ctypes.c_int64 * len(_abi.PHASES))()
    ctx.check(ctx.lib.lv_read_timings(ctx.h, ctypes.cast(ms, ctypes.c_void_p),
                                      ctypes.cast(calls, ctypes.c_void_p)), "lv_read_timings")
    return {name: (ms[i], calls[i]) for i, name in enumerate(_abi.PHASES)}


# -------------------------------------------------------- convenience layer

class Renderer:
    """Owns the scratch workspace and a default saved-state buffer of one
    (voxels, frame, settings) shape, and re-plans the pair capacity when
    lv_check_overflow reports an overflow.  A forward pass writes its saved
    state into `saved` (the renderer's own when None); the backward of that
    pass must be given the same buffer and the settings the pass ran with."""

    def __init__(self, ctx: Context, vox: Voxels, frame: Frame, st: Optional[LvSettings] = None):
        self.ctx, self.vox, self.frame = ctx, vox, frame
        self.st = st if st is not None else settings()
        if self.st.pair_capacity == 0:
            self.st.pair_capacity = min(max(1 << 20, (3 * vox.n * frame.n_views) // 2), (1 << 32) - 1)
        self._alloc()
        self.checked = False

    def _alloc(self):
        ws, sv = query_sizes(self.ctx, self.vox, self.frame, self.st)
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=self.ctx.device)
        self.saved_bytes = sv
        self.saved = self.new_saved()

    def new_saved(self) -> torch.Tensor:
        """A fresh buffer for the saved state of one forward pass."""
        return torch.empty(self.saved_bytes, dtype=torch.uint8, device=self.ctx.device)

    def settings_copy(self) -> LvSettings:
        return LvSettings.from_buffer_copy(self.st)

    def new_outputs(self):
        d = self.ctx.device
        P = self.frame.P
        return (torch.empty(3 * P, device=d), torch.empty(P, device=d), torch.empty(P, device=d))

    def forward(self, rgb, depth, alpha, wmax, vox: Optional[Voxels] = None, stream=None,
                verify: Optional[bool] = None, saved: Optional[torch.Tensor] = None,
                dist: Optional[torch.Tensor] = None, normal: Optional[torch.Tensor] = None,
                mdepth: Optional[torch.Tensor] = None):
        """Returns the saved-state buffer the pass wrote (`saved`, or a larger
        replacement after a capacity re-plan; the renderer's own if None).
        With dist, normal and/or mdepth the pass also renders those channels
        (lv_forward_aux)."""
        vox = vox or self.vox
        own = saved is None
        saved = self.saved if own else saved
        verify = verify or (verify is None and not self.checked)
        # a truncated pass composites without some occluders, so its weights
        # are not bounded by the true ones: keep w_max to restore on overflow
        keep = wmax.clone() if (verify and wmax is not None) else None
        aux = dist is not None or normal is not None or mdepth is not None

        def run(sv):
            if aux:
                forward_aux(self.ctx, vox, self.frame, self.st, self.workspace, sv, rgb, depth,
                            alpha, wmax, dist, normal, mdepth, stream)
            else:
                forward(self.ctx, vox, self.frame, self.st, self.workspace, sv, rgb, depth, alpha,
                        wmax, stream)

        run(saved)
        if verify:
            fits, need = check_overflow(self.ctx, vox, self.frame, self.st, saved, stream)
            self.checked = True
            if not fits:
                if keep is not None:
                    wmax.copy_(keep)
                self.st.pair_capacity = min(need + need // 8 + 4096, (1 << 32) - 1)
                self._alloc()
                saved = self.saved if own else self.new_saved()
                run(saved)
                fits, need = check_overflow(self.ctx, vox, self.frame, self.st, saved, stream)
                if not fits:
                    raise LiteVoxelError(_abi.LV_ERR_CAPACITY, f"{need} pairs do not fit")
        return saved

    def backward(self, d_rgb, d_depth, d_alpha, d_density, d_sh, vox: Optional[Voxels] = None,
                 stream=None, saved: Optional[torch.Tensor] = None, st: Optional[LvSettings] = None):
        """saved/st: the buffer and settings of the forward pass being
        differentiated (default: the renderer's own)."""
        st = st if st is not None else self.st
        saved = self.saved if saved is None else saved
        ws, _ = query_sizes(self.ctx, vox or self.vox, self.frame, st)
        if ws > self.workspace.numel():
            raise LiteVoxelError(_abi.LV_ERR_ARG, "workspace smaller than the pass needs")
        backward(self.ctx, vox or self.vox, self.frame, st, self.workspace, saved, d_rgb, d_depth,
                 d_alpha, d_density, d_sh, stream)

    def backward_aux(self, d_rgb, d_depth, d_alpha, depth_fwd, d_dist, d_normal, d_density, d_sh,
                     vox: Optional[Voxels] = None, stream=None,
                     saved: Optional[torch.Tensor] = None, st: Optional[LvSettings] = None):
        """backward() with the upstream gradients of the distortion and normal
        channels (lv_backward_aux); depth_fwd: the depth the pass rendered."""
        st = st if st is not None else self.st
        saved = self.saved if saved is None else saved
        ws, _ = query_sizes(self.ctx, vox or self.vox, self.frame, st)
        if ws > self.workspace.numel():
            raise LiteVoxelError(_abi.LV_ERR_ARG, "workspace smaller than the pass needs")
        backward_aux(self.ctx, vox or self.vox, self.frame, st, self.workspace, saved, d_rgb,
                     d_depth, d_alpha, depth_fwd, d_dist, d_normal, d_density, d_sh, stream)


class RasterizeFn(torch.autograd.Function):
    """(density [8,N] or [n_grid] in the renderer's layout, sh [K,N]) ->
    (rgb [3P], depth [P], alpha [P]); gradients with respect to the stored
    density values (through the layout's activation) and the SH.

    Every forward pass gets a saved-state buffer of its own (tile lists,
    records and the per-pixel index of the last hit with the transmittance
    before it), kept on the autograd node with the settings it ran with, so
    several passes on one renderer can be differentiated in any order.  The
    backward recomputes transmittance back to front inside lv_backward from
    that state: no per-sample state is kept.  w_max is max-accumulated into
    `wmax` (not differentiable).
    """

    @staticmethod
    def forward(ctx, density, sh, renderer: Renderer, wmax: torch.Tensor):
        vox = renderer.vox.with_params(density.detach().contiguous(), sh.detach().contiguous())
        rgb, depth, alpha = renderer.new_outputs()
        saved = renderer.forward(rgb, depth, alpha, wmax, vox=vox, saved=renderer.new_saved())
        ctx.renderer = renderer
        ctx.vox = vox
        ctx.saved_state = saved
        ctx.st = renderer.settings_copy()
        ctx.mark_non_differentiable(wmax)
        return rgb, depth, alpha

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_alpha):
        r = ctx.renderer
        vox = ctx.vox
        d_density = torch.empty_like(vox.density)
        d_sh = torch.empty_like(vox.sh)
        g_rgb = g_rgb.contiguous() if g_rgb is not None else torch.zeros(3 * r.frame.P, device=vox.density.device)
        g_depth = g_depth.contiguous() if g_depth is not None else None
        g_alpha = g_alpha.contiguous() if g_alpha is not None else None
        r.backward(g_rgb, g_depth, g_alpha, d_density, d_sh, vox=vox, saved=ctx.saved_state,
                   st=ctx.st)
        return d_density, d_sh, None, None


def rasterize(density, sh, renderer: Renderer, wmax: torch.Tensor):
    return RasterizeFn.apply(density, sh, renderer, wmax)


class RasterizeAuxFn(torch.autograd.Function):
    """RasterizeFn with the auxiliary channels: (density, sh) -> (rgb [3P],
    depth [P], alpha [P], dist [P], normal [3P], mdepth [P]; mdepth is not
    differentiable).  The node keeps the pass's saved state and its depth
    (the backward of the distortion reads it)."""

    @staticmethod
    def forward(ctx, density, sh, renderer: Renderer, wmax: torch.Tensor):
        vox = renderer.vox.with_params(density.detach().contiguous(), sh.detach().contiguous())
        rgb, depth, alpha = renderer.new_outputs()
        P = renderer.frame.P
        dist = torch.empty(P, device=rgb.device)
        normal = torch.empty(3 * P, device=rgb.device)
        mdepth = torch.empty(P, device=rgb.device)
        saved = renderer.forward(rgb, depth, alpha, wmax, vox=vox, saved=renderer.new_saved(),
                                 dist=dist, normal=normal, mdepth=mdepth)
        ctx.renderer, ctx.vox, ctx.saved_state = renderer, vox, saved
        ctx.st = renderer.settings_copy()
        ctx.depth = depth.detach().clone()
        ctx.mark_non_differentiable(wmax, mdepth)
        return rgb, depth, alpha, dist, normal, mdepth

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_alpha, g_dist, g_normal, g_mdepth):
        r, vox = ctx.renderer, ctx.vox
        d_density = torch.empty_like(vox.density)
        d_sh = torch.empty_like(vox.sh)
        c = lambda g: g.contiguous() if g is not None else None
        g_rgb = c(g_rgb) if g_rgb is not None else torch.zeros(3 * r.frame.P, device=vox.density.device)
        r.backward_aux(g_rgb, c(g_depth), c(g_alpha), ctx.depth, c(g_dist), c(g_normal), d_density,
                       d_sh, vox=vox, saved=ctx.saved_state, st=ctx.st)
        return d_density, d_sh, None, None


def rasterize_aux(density, sh, renderer: Renderer, wmax: torch.Tensor):
    return RasterizeAuxFn.apply(density, sh, renderer, wmax)
