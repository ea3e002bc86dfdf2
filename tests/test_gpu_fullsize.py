"""Parity at the benchmark's full size (1M voxels, SH3, 8 ring views of uneven
resolution, 9.37 MP) in the launch configuration the benchmark picks with the
autotuner.  The oracle computes what it can one by one: every record's key and
every tile list (bit-exact), a seeded sample of pixels, w_max of a sample of
voxels (over every pixel their footprint covers), and the gradient of a loss
whose upstream gradient lives on the sampled pixels only."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import GRAD_TOL, IMG_TOL, WMAX_TOL, rel_l2, rgb_index, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_02510_amd as lv
    c = lv.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ring(ctx):
    import paper_2511_02510_amd as lv
    import torch
    say("full size: generating the 1M-voxel ring workload")
    scene, cams, _ = synth.make_config("ring1m")
    dev = ctx.device
    vox = lv.Voxels.from_scene(scene, dev)
    frame = lv.Frame(cams, dev)
    best, table = lv.autotune(ctx, vox, frame, reps=2)
    say(f"  autotuned tile={best.tile} chunk={best.chunk}")
    rng = np.random.default_rng(2511)
    P = frame.P
    pix = np.sort(rng.choice(P, size=4000, replace=False))
    g_rgb = np.zeros(3 * P)
    g_rgb[rgb_index(cams, pix)] = rng.normal(0, 1e-2, 3 * pix.shape[0])
    g_depth = np.zeros(P)
    g_depth[pix] = rng.normal(0, 1e-3, pix.shape[0])
    g_alpha = np.zeros(P)
    g_alpha[pix] = rng.normal(0, 1e-2, pix.shape[0])
    r = lv.Renderer(ctx, vox, frame, lv.settings(tile=best.tile, chunk=best.chunk,
                                                 pair_capacity=best.pair_capacity))
    rgb, depth, alpha = r.new_outputs()
    wmax = torch.zeros(vox.n, device=dev)
    r.forward(rgb, depth, alpha, wmax)
    dd = torch.empty_like(vox.density)
    dsh = torch.empty_like(vox.sh)
    r.backward(to_dev(g_rgb, dev), to_dev(g_depth, dev), to_dev(g_alpha, dev), dd, dsh)
    torch.cuda.synchronize()
    out = dict(scene=scene, cams=cams, pix=pix, grads=(g_rgb, g_depth, g_alpha), tile=best.tile,
               rgb=rgb.cpu().numpy().astype(np.float64), depth=depth.cpu().numpy().astype(np.float64),
               alpha=alpha.cpu().numpy().astype(np.float64), wmax=wmax.cpu().numpy().astype(np.float64),
               dd=dd.cpu().numpy().astype(np.float64), dsh=dsh.cpu().numpy().astype(np.float64),
               bins=lv.export_bins(ctx, vox, frame, r.st, r.saved))
    return out


def test_fullsize_keys_and_tile_lists_bit_exact(ring):
    say("full size: keys and per-tile order")
    scene, cams, b = ring["scene"], ring["cams"], ring["bins"]
    vis, rect, code = oracle.project_keys(scene, cams)
    assert np.array_equal(b["vis"], vis)
    on = vis == 1
    assert np.array_equal(b["rects"][on], rect[on])
    assert np.array_equal(b["codes"][on], code[on])
    start, ids, _ = oracle.tile_lists(cams, vis, rect, code, ring["tile"])
    assert np.array_equal(b["tile_start"], start)
    assert np.array_equal(b["ids"], ids)
    say(f"  {int(on.sum())} records, {ids.shape[0]} pairs identical")


def test_fullsize_sampled_pixels(ring):
    say("full size: 4000 sampled pixels")
    ref = oracle.render(ring["scene"], ring["cams"], pix_list=ring["pix"])
    pix = ring["pix"]
    idx = rgb_index(ring["cams"], pix)
    e_rgb = np.abs(ring["rgb"][idx] - ref["rgb"][idx]).max()
    e_d = np.abs(ring["depth"][pix] - ref["depth"][pix]).max()
    e_a = np.abs(ring["alpha"][pix] - ref["alpha"][pix]).max()
    say(f"  max abs: rgb {e_rgb:.2e} depth {e_d:.2e} alpha {e_a:.2e}")
    assert e_rgb <= IMG_TOL and e_d <= IMG_TOL and e_a <= IMG_TOL


def test_fullsize_sampled_wmax(ring):
    say("full size: w_max of 200 sampled voxels")
    scene, cams = ring["scene"], ring["cams"]
    vis, _, _ = oracle.project_keys(scene, cams)
    seen = np.nonzero(vis.any(axis=0))[0]
    rng = np.random.default_rng(7)
    vsel = np.sort(rng.choice(seen, size=200, replace=False))
    fp = oracle.footprint_pixels(scene, cams, vsel)
    ref = oracle.render(scene, cams, pix_list=fp)
    e = np.abs(ring["wmax"][vsel] - ref["wmax"][vsel]).max()
    say(f"  {fp.shape[0]} footprint pixels, max abs {e:.2e}")
    assert e <= WMAX_TOL
    assert np.count_nonzero(ref["wmax"][vsel]) > 100


def test_fullsize_gradient_of_sampled_pixels(ring):
    say("full size: gradient of a loss on the sampled pixels")
    dd, dsh = oracle.backward(ring["scene"], ring["cams"], *ring["grads"], pix_list=ring["pix"])
    e1, e2 = rel_l2(ring["dd"], dd), rel_l2(ring["dsh"], dsh)
    say(f"  rel L2: density {e1:.2e} sh {e2:.2e}")
    assert e1 <= GRAD_TOL and e2 <= GRAD_TOL
    assert np.count_nonzero(dd) > 1000
