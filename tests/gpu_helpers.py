"""Shared helpers of the GPU parity tests: run the HIP path through the C-ABI
binding and compare with the oracle on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np

import oracle
import synth

IMG_TOL = 1e-4      # rgb / depth / alpha, max abs (FP32 GPU vs FP64 oracle)
WMAX_TOL = 1e-5     # w_max, max abs
GRAD_TOL = 1e-3     # gradients, relative L2


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def lv():
    import paper_2511_02510_amd as m
    return m


def to_dev(a, dev, dtype=np.float32):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to(dev)


def run_gpu(ctx, scene, cams, tile=16, chunk=64, bg=(0.0, 0.0, 0.0), cap=0, grads=None,
            export=True, wmax_in=None, chunk_bwd=0):
    """Forward (+ backward when grads = (g_rgb, g_depth, g_alpha)) on the GPU."""
    import torch
    m = lv()
    dev = ctx.device
    vox = m.Voxels.from_scene(scene, dev)
    frame = m.Frame(cams, dev, bg)
    r = m.Renderer(ctx, vox, frame, m.settings(tile=tile, chunk=chunk, pair_capacity=cap,
                                               chunk_bwd=chunk_bwd))
    rgb, depth, alpha = r.new_outputs()
    wmax = torch.zeros(max(vox.n, 1), device=dev) if wmax_in is None else to_dev(wmax_in, dev)
    r.forward(rgb, depth, alpha, wmax)
    out = {}
    if grads is not None:
        g_rgb, g_depth, g_alpha = grads
        dd = torch.empty_like(vox.density)
        dsh = torch.empty_like(vox.sh)
        r.backward(to_dev(g_rgb, dev), None if g_depth is None else to_dev(g_depth, dev),
                   None if g_alpha is None else to_dev(g_alpha, dev), dd, dsh)
        out["dd"] = dd.cpu().numpy().astype(np.float64)
        out["dsh"] = dsh.cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    out.update(rgb=rgb.cpu().numpy().astype(np.float64), depth=depth.cpu().numpy().astype(np.float64),
               alpha=alpha.cpu().numpy().astype(np.float64),
               wmax=wmax.cpu().numpy().astype(np.float64)[:vox.n])
    if export:
        out["bins"] = m.export_bins(ctx, vox, frame, r.st, r.saved)
    out["renderer"] = r
    return out


def check_keys(gpu_bins, scene, cams, tile):
    """Keys and per-tile order bit-exact against the oracle's binary32 key path."""
    vis, rect, code = oracle.project_keys(scene, cams)
    assert np.array_equal(gpu_bins["vis"], vis), "visibility"
    on = vis == 1
    assert np.array_equal(gpu_bins["rects"][on], rect[on]), "pixel-centre ranges"
    assert np.array_equal(gpu_bins["codes"][on], code[on]), "visibility codes"
    start, ids, keys = oracle.tile_lists(cams, vis, rect, code, tile)
    assert np.array_equal(gpu_bins["tile_start"], start), "tile ranges"
    assert np.array_equal(gpu_bins["ids"], ids), "per-tile order"
    return int(start[-1])


def check_images(gpu, ref, pix=None, cams=None):
    """Max-abs image errors over all pixels, or over global pixel indices pix
    (cams then gives the per-view rgb layout)."""
    if pix is None:
        e_rgb = np.abs(gpu["rgb"] - ref["rgb"]).max(initial=0.0)
        e_d = np.abs(gpu["depth"] - ref["depth"]).max(initial=0.0)
        e_a = np.abs(gpu["alpha"] - ref["alpha"]).max(initial=0.0)
    else:
        e_d = np.abs(gpu["depth"][pix] - ref["depth"][pix]).max(initial=0.0)
        e_a = np.abs(gpu["alpha"][pix] - ref["alpha"][pix]).max(initial=0.0)
        idx = rgb_index(cams, pix)
        e_rgb = np.abs(gpu["rgb"][idx] - ref["rgb"][idx]).max(initial=0.0)
    say(f"  max abs: rgb {e_rgb:.2e} depth {e_d:.2e} alpha {e_a:.2e}")
    assert e_rgb <= IMG_TOL and e_d <= IMG_TOL and e_a <= IMG_TOL
    return e_rgb, e_d, e_a


def rgb_index(cams, pix):
    """Flat rgb indices (3 per pixel) of global pixel indices."""
    off = oracle.pix_offsets(cams)
    v = np.searchsorted(off, pix, side="right") - 1
    local = pix - off[v]
    npv = off[v + 1] - off[v]
    base = 3 * off[v] + local
    return np.concatenate([base, base + npv, base + 2 * npv])


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def random_grads(rng, P, scale=1e-3):
    return (rng.normal(0, scale, 3 * P), rng.normal(0, scale * 0.1, P), rng.normal(0, scale, P))


def small_shell(n, seed, deg=3, lmin=5, lmax=8, clutter=0.0):
    rng = np.random.default_rng(seed)
    return synth.make_scene_shell(rng, n, lmin, lmax, sh_degree=deg, clutter_frac=clutter)
