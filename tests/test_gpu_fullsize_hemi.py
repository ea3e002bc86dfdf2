"""Parity on the large training-step workload: 4M octree leaves (levels 8-12),
SH3, 16 views of 1920x1080 on a hemisphere (33.2 MP), with the depth-binned
w_max quantile (16 bins, q = 0.1) on device.  The oracle computes what it can
one by one: every record's key and every tile list (bit-exact), a seeded
sample of pixels, every pixel of two whole views (each view's image depends
on that view only), w_max of a sample of voxels (over every pixel their
footprint covers), the gradient of a loss that lives on the sampled pixels
and of one on every pixel of the two views, and the bins, cutoffs and prune
mask from the GPU's own w_max (bit-exact)."""
import numpy as np
import pytest

import oracle
from oracle import quantile as oquant
import synth
from gpu_helpers import GRAD_TOL, IMG_TOL, WMAX_TOL, rel_l2, rgb_index, say, to_dev

pytestmark = pytest.mark.gpu

TILE, CHUNK = 16, 128
WHOLE = (3, 11)   # views compared pixel by pixel


@pytest.fixture(scope="module")
def hemi():
    import paper_2511_02510_amd as lv
    import torch
    ctx = lv.Context(0)
    say("hemisphere: generating the 4M-voxel, 16-view workload")
    scene, cams, _ = synth.make_config("hemi4m")
    dev = ctx.device
    vox = lv.Voxels.from_scene(scene, dev)
    frame = lv.Frame(cams, dev)
    rng = np.random.default_rng(2512)
    P = frame.P
    pix = np.sort(rng.choice(P, size=4000, replace=False))
    g_rgb = np.zeros(3 * P)
    g_rgb[rgb_index(cams, pix)] = rng.normal(0, 1e-2, 3 * pix.shape[0])
    g_depth = np.zeros(P)
    g_depth[pix] = rng.normal(0, 1e-3, pix.shape[0])
    g_alpha = np.zeros(P)
    g_alpha[pix] = rng.normal(0, 1e-2, pix.shape[0])
    r = lv.Renderer(ctx, vox, frame, lv.settings(tile=TILE, chunk=CHUNK))
    rgb, depth, alpha = r.new_outputs()
    wmax = torch.zeros(vox.n, device=dev)
    say("  forward + backward")
    r.forward(rgb, depth, alpha, wmax)
    dd = torch.empty_like(vox.density)
    dsh = torch.empty_like(vox.sh)
    r.backward(to_dev(g_rgb, dev), to_dev(g_depth, dev), to_dev(g_alpha, dev), dd, dsh)
    nb = 16
    ws = torch.empty(lv.quantile_workspace_size(vox.n, nb), dtype=torch.uint8, device=dev)
    tau = torch.empty(nb, device=dev)
    prune = torch.empty(vox.n, dtype=torch.uint8, device=dev)
    bins = torch.empty(vox.n, dtype=torch.uint8, device=dev)
    lv.depth_quantile(ctx, vox, frame, wmax, nb, 0.1, ws, tau, prune, bins)
    # a loss on every pixel of the two whole views
    off = oracle.pix_offsets(cams)
    w_rgb, w_depth = np.zeros(3 * P), np.zeros(P)
    for v in WHOLE:
        n = int(off[v + 1] - off[v])
        w_rgb[3 * int(off[v]):3 * int(off[v + 1])] = rng.normal(0, 1e-3, 3 * n)
        w_depth[int(off[v]):int(off[v + 1])] = rng.normal(0, 1e-4, n)
    ddw = torch.empty_like(vox.density)
    dshw = torch.empty_like(vox.sh)
    say("  backward of a loss on two whole views")
    r.backward(to_dev(w_rgb, dev), to_dev(w_depth, dev), None, ddw, dshw)
    torch.cuda.synchronize()
    say("  exporting the tile lists")
    out = dict(scene=scene, cams=cams, pix=pix, grads=(g_rgb, g_depth, g_alpha),
               rgb=rgb.cpu().numpy().astype(np.float64), depth=depth.cpu().numpy().astype(np.float64),
               alpha=alpha.cpu().numpy().astype(np.float64), wmax=wmax.cpu().numpy(),
               dd=dd.cpu().numpy().astype(np.float64), dsh=dsh.cpu().numpy().astype(np.float64),
               bins=bins.cpu().numpy(), tau=tau.cpu().numpy(), prune=prune.cpu().numpy(),
               wgrads=(w_rgb, w_depth), ddw=ddw.cpu().numpy().astype(np.float64),
               dshw=dshw.cpu().numpy().astype(np.float64),
               tiles=lv.export_bins(ctx, vox, frame, r.st, r.saved))
    del r, vox, frame
    ctx.close()
    return out


def test_hemi_keys_and_tile_lists_bit_exact(hemi):
    say("hemisphere: keys and per-tile order")
    scene, cams, b = hemi["scene"], hemi["cams"], hemi["tiles"]
    vis, rect, code = oracle.project_keys(scene, cams)
    assert np.array_equal(b["vis"], vis)
    on = vis == 1
    assert np.array_equal(b["rects"][on], rect[on])
    assert np.array_equal(b["codes"][on], code[on])
    start, ids, _ = oracle.tile_lists(cams, vis, rect, code, TILE)
    assert np.array_equal(b["tile_start"], start)
    assert np.array_equal(b["ids"], ids)
    say(f"  {int(on.sum())} records, {ids.shape[0]} pairs identical")


def test_hemi_sampled_pixels(hemi):
    say("hemisphere: 4000 sampled pixels")
    ref = oracle.render(hemi["scene"], hemi["cams"], pix_list=hemi["pix"])
    pix = hemi["pix"]
    idx = rgb_index(hemi["cams"], pix)
    e_rgb = np.abs(hemi["rgb"][idx] - ref["rgb"][idx]).max()
    e_d = np.abs(hemi["depth"][pix] - ref["depth"][pix]).max()
    e_a = np.abs(hemi["alpha"][pix] - ref["alpha"][pix]).max()
    say(f"  max abs: rgb {e_rgb:.2e} depth {e_d:.2e} alpha {e_a:.2e}")
    assert e_rgb <= IMG_TOL and e_d <= IMG_TOL and e_a <= IMG_TOL


def _views(hemi, flat3, flat1):
    """The two whole views' rgb and depth/alpha slices of full-frame arrays."""
    off = oracle.pix_offsets(hemi["cams"])
    rgb = np.concatenate([flat3[3 * int(off[v]):3 * int(off[v + 1])] for v in WHOLE])
    one = [np.concatenate([a[int(off[v]):int(off[v + 1])] for v in WHOLE]) for a in flat1]
    return rgb, one


def test_hemi_two_whole_views_every_pixel(hemi):
    say(f"hemisphere: every pixel of views {WHOLE} (2 x 1920 x 1080)")
    sub = [hemi["cams"][v] for v in WHOLE]
    ref = oracle.render(hemi["scene"], sub)
    rgb, (depth, alpha) = _views(hemi, hemi["rgb"], (hemi["depth"], hemi["alpha"]))
    e_rgb = np.abs(rgb - ref["rgb"]).max()
    e_d = np.abs(depth - ref["depth"]).max()
    e_a = np.abs(alpha - ref["alpha"]).max()
    say(f"  max abs: rgb {e_rgb:.2e} depth {e_d:.2e} alpha {e_a:.2e}")
    assert e_rgb <= IMG_TOL and e_d <= IMG_TOL and e_a <= IMG_TOL
    assert np.count_nonzero(ref["alpha"]) > 100000


def test_hemi_two_whole_views_gradient(hemi):
    say(f"hemisphere: gradient of a loss on every pixel of views {WHOLE}")
    sub = [hemi["cams"][v] for v in WHOLE]
    g_rgb, (g_depth,) = _views(hemi, hemi["wgrads"][0], (hemi["wgrads"][1],))
    dd, dsh = oracle.backward(hemi["scene"], sub, g_rgb, g_depth)
    e1, e2 = rel_l2(hemi["ddw"], dd), rel_l2(hemi["dshw"], dsh)
    say(f"  rel L2: density {e1:.2e} sh {e2:.2e}")
    assert e1 <= GRAD_TOL and e2 <= GRAD_TOL


def test_hemi_sampled_wmax(hemi):
    say("hemisphere: w_max of 100 sampled voxels")
    scene, cams = hemi["scene"], hemi["cams"]
    seen = np.nonzero(hemi["tiles"]["vis"].any(axis=0))[0]
    rng = np.random.default_rng(8)
    vsel = np.sort(rng.choice(seen, size=100, replace=False))
    fp = oracle.footprint_pixels(scene, cams, vsel)
    ref = oracle.render(scene, cams, pix_list=fp)
    e = np.abs(hemi["wmax"][vsel].astype(np.float64) - ref["wmax"][vsel]).max()
    say(f"  {fp.shape[0]} footprint pixels, max abs {e:.2e}")
    assert e <= WMAX_TOL
    assert np.count_nonzero(ref["wmax"][vsel]) > 50


def test_hemi_gradient_of_sampled_pixels(hemi):
    say("hemisphere: gradient of a loss on the sampled pixels")
    dd, dsh = oracle.backward(hemi["scene"], hemi["cams"], *hemi["grads"], pix_list=hemi["pix"])
    e1, e2 = rel_l2(hemi["dd"], dd), rel_l2(hemi["dsh"], dsh)
    say(f"  rel L2: density {e1:.2e} sh {e2:.2e}")
    assert e1 <= GRAD_TOL and e2 <= GRAD_TOL
    assert np.count_nonzero(dd) > 1000


def test_hemi_depth_quantile_bit_exact_on_same_wmax(hemi):
    say("hemisphere: depth bins, cutoffs and prune mask over 4M voxels")
    ref = oquant.depth_quantile(hemi["scene"], hemi["cams"], hemi["wmax"].astype(np.float32), 16, 0.1)
    assert np.array_equal(hemi["bins"], ref["bins"])
    assert np.array_equal(hemi["tau"], ref["tau"])
    assert np.array_equal(hemi["prune"], ref["prune"])
    counts = np.bincount(ref["bins"], minlength=16)
    say(f"  bin sizes {counts.tolist()}, pruned {int(ref['prune'].sum())}")
    assert (counts > 0).sum() >= 8
