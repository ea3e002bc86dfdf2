"""Parity on the 200,000-leaf SH-3 shell (octree levels 6-10) seen by one
800 x 600 camera, in the benchmark's launch configuration (tile 16, forward
chunk 128, backward chunk 64): the forward with w_max (keys and tile lists
bit-exact, every pixel, every voxel), then fwd+bwd through the real loss chain
-- the ramped inverse-Sobel weight w = (1 + g/g99)^-gamma at the ramp's ends
and middle, the weighted L1 of eq. 10 and its image gradient, the backward --
against the oracle's chain, over the whole gradient.  Also the same leaves
stored in a shuffled order on a 1600 x 1080 view at tile 8, where a block of
consecutive leaves spans far more tiles than its LDS table holds (the direct
per-tile counting and emission paths of the binning)."""
import numpy as np
import pytest

import oracle
from oracle import loss as oloss
import synth
from synth.scenes import look_at
from gpu_helpers import (GRAD_TOL, IMG_TOL, WMAX_TOL, check_keys, rel_l2, say, to_dev)

pytestmark = pytest.mark.gpu

TILE, CHUNK, CHUNK_BWD = 16, 128, 64


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_02510_amd as lv
    c = lv.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def shell():
    say("shell200k: generating the scene and its oracle image")
    scene, cams, targets = synth.make_config("shell200k_train")
    return dict(scene=scene, cams=cams, targets=targets, ref=oracle.render(scene, cams))


def _run_chain(ctx, scene, cams, targets, gamma, tile=TILE, chunk=CHUNK, chunk_bwd=CHUNK_BWD,
               form=1):
    import paper_2511_02510_amd as lv
    import torch
    dev = ctx.device
    vox = lv.Voxels.from_scene(scene, dev)
    frame = lv.Frame(cams, dev)
    r = lv.Renderer(ctx, vox, frame, lv.settings(tile=tile, chunk=chunk, chunk_bwd=chunk_bwd))
    rgb, depth, alpha = r.new_outputs()
    wmax = torch.zeros(vox.n, device=dev)
    target = to_dev(np.concatenate([t.ravel() for t in targets]), dev)
    weight = torch.empty(frame.P, device=dev)
    lw_ws = torch.empty(lv.lf_weight_workspace_size(frame.n_views), dtype=torch.uint8, device=dev)
    loss = torch.empty(frame.n_views, device=dev)
    d_rgb = torch.empty(3 * frame.P, device=dev)
    dd = torch.empty_like(vox.density)
    dsh = torch.empty_like(vox.sh)
    r.forward(rgb, depth, alpha, wmax)
    lv.lf_weight(ctx, frame, target, gamma, form, 1e-3, weight, lw_ws)
    lv.l1_grad(ctx, frame, rgb, target, weight, loss, d_rgb)
    r.backward(d_rgb, None, None, dd, dsh)
    torch.cuda.synchronize()
    f64 = lambda t: t.cpu().numpy().astype(np.float64)
    return dict(rgb=f64(rgb), depth=f64(depth), alpha=f64(alpha), wmax=f64(wmax),
                loss=f64(loss), d_rgb=f64(d_rgb), dd=f64(dd), dsh=f64(dsh),
                bins=lv.export_bins(ctx, vox, frame, r.st, r.saved))


def _check_forward(g, ref, what):
    e_rgb = np.abs(g["rgb"] - ref["rgb"]).max()
    e_d = np.abs(g["depth"] - ref["depth"]).max()
    e_a = np.abs(g["alpha"] - ref["alpha"]).max()
    e_w = np.abs(g["wmax"] - ref["wmax"]).max()
    say(f"  {what}: max abs rgb {e_rgb:.2e} depth {e_d:.2e} alpha {e_a:.2e} w_max {e_w:.2e}")
    assert e_rgb <= IMG_TOL and e_d <= IMG_TOL and e_a <= IMG_TOL
    assert e_w <= WMAX_TOL


def _check_chain(g, scene, cams, targets, views, gamma, form=1):
    grads, losses = [], []
    for v in range(len(cams)):
        w = oloss.lf_weight(targets[v], gamma, form=form, eps=1e-3)
        l, gr = oloss.l1_loss_grad(views[v], targets[v], w)
        losses.append(l)
        grads.append(gr)
    g_ref = oracle.join_views(grads)
    e_l = float(np.max(np.abs(g["loss"] - np.array(losses)) / np.abs(np.array(losses))))
    flip = np.sign(g["d_rgb"]) != np.sign(g_ref)
    dd, dsh = oracle.backward(scene, cams, g_ref)
    e1, e2 = rel_l2(g["dd"], dd), rel_l2(g["dsh"], dsh)
    say(f"  loss max rel {e_l:.2e}, {int(flip.sum())} L1 signs differ, "
        f"rel L2 density {e1:.2e} sh {e2:.2e}")
    assert e_l <= 1e-5
    assert flip.sum() <= max(3, 1e-5 * flip.size)
    assert e1 <= GRAD_TOL and e2 <= GRAD_TOL
    assert np.count_nonzero(dd) > 50000


def test_shell200k_forward_keys_pixels_wmax(ctx, shell):
    say("shell200k: forward + w_max (keys, every pixel, every voxel)")
    g = _run_chain(ctx, shell["scene"], shell["cams"], shell["targets"], 0.0)
    Q = check_keys(g["bins"], shell["scene"], shell["cams"], TILE)
    say(f"  {Q} pairs identical")
    _check_forward(g, shell["ref"], "all pixels / voxels")
    assert np.count_nonzero(shell["ref"]["wmax"]) > 100000


@pytest.mark.parametrize("gamma", [0.0, 0.5, 1.0])
def test_shell200k_loss_chain_gradient(ctx, shell, gamma):
    say(f"shell200k: fwd+bwd through the loss chain, gamma {gamma}")
    g = _run_chain(ctx, shell["scene"], shell["cams"], shell["targets"], gamma)
    _check_chain(g, shell["scene"], shell["cams"], shell["targets"], shell["ref"]["views"], gamma)


def test_shuffled_leaves_wide_view_tile8(ctx, shell):
    say("shuffled leaf order, 1600 x 1080, tile 8 (direct binning paths)")
    rng = np.random.default_rng(251102519)
    sc = synth.scene_subset(shell["scene"], rng.permutation(shell["scene"].n)[:120000])
    cams = [look_at((1.4, 0.9, 1.9), 1600, 1080)]
    targets = [synth.make_target(rng, 1600, 1080)]
    g = _run_chain(ctx, sc, cams, targets, 0.5, tile=8, chunk=64, chunk_bwd=64)
    Q = check_keys(g["bins"], sc, cams, 8)
    say(f"  {Q} pairs identical")
    ref = oracle.render(sc, cams)
    _check_forward(g, ref, "all pixels / voxels")
    _check_chain(g, sc, cams, targets, ref["views"], 0.5)
