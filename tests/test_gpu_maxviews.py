"""The largest frame the C-ABI takes (LV_MAX_VIEWS = 256 views of small,
uneven sizes) through every entry point with per-view state, against the
FP64 oracle: keys, images, w_max and gradients of the rasterizer (the view
of every tile, per-view tile and pixel offsets, queues over many views), the
auxiliary channels and terms (per-view tile offsets of the terms kernel),
the loss weight and L1 gradient (per-view normalisation and loss sums) and
the depth quantile (the proxy's minimum over all views)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import aux as oaux
from oracle import loss as oloss
from oracle import quantile as oquant
from synth.scenes import look_at
from gpu_helpers import (GRAD_TOL, IMG_TOL, WMAX_TOL, check_images, check_keys, random_grads,
                         rel_l2, run_gpu, say, small_shell, to_dev)

pytestmark = pytest.mark.gpu

N_VIEWS = 256


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_02510_amd as lv
    c = lv.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def problem():
    import paper_2511_02510_amd._abi as abi
    assert abi.LV_MAX_VIEWS == N_VIEWS
    scene = small_shell(6000, seed=151, deg=2, lmin=4, lmax=7, clutter=0.2)
    rng = np.random.default_rng(152)
    cams = []
    for i in range(N_VIEWS):
        # generic directions (no camera on a coordinate plane) on a sphere
        # of views, sizes 3..24 x 2..19 so most tiles are ragged
        az = 2 * np.pi * i / N_VIEWS * 7.0 + 0.137
        el = 1.2 * np.sin(0.31 * i + 0.2) + 0.071
        r = 2.2 + 0.5 * np.cos(0.17 * i)
        o = r * np.array([np.cos(el) * np.cos(az), np.sin(el), np.cos(el) * np.sin(az)])
        cams.append(look_at(tuple(o), int(rng.integers(3, 25)), int(rng.integers(2, 20))))
    return scene, cams


def test_max_views_forward_backward_and_keys(ctx, problem):
    scene, cams = problem
    P = sum(c.npix for c in cams)
    say(f"{N_VIEWS} views, {P} px: keys, forward, backward")
    grads = random_grads(np.random.default_rng(153), P)
    ref = oracle.render(scene, cams)
    dd, dsh = oracle.backward(scene, cams, *grads)
    for tile in (8, 16):
        g = run_gpu(ctx, scene, cams, tile=tile, chunk=64, grads=grads)
        check_keys(g["bins"], scene, cams, tile)
        check_images(g, ref)
        assert np.abs(g["wmax"] - ref["wmax"]).max() <= WMAX_TOL
        e1, e2 = rel_l2(g["dd"], dd), rel_l2(g["dsh"], dsh)
        say(f"  tile {tile}: gradient rel-L2 density {e1:.2e} sh {e2:.2e}")
        assert e1 <= GRAD_TOL and e2 <= GRAD_TOL


def test_max_views_aux_channels_and_terms(ctx, problem):
    import torch
    import paper_2511_02510_amd as lv
    scene, cams = problem
    dev = ctx.device
    vox = lv.Voxels.from_scene(scene, dev)
    frame = lv.Frame(cams, dev)
    P = frame.P
    r = lv.Renderer(ctx, vox, frame, lv.settings(tile=16, chunk=64))
    rgb, depth, alpha = r.new_outputs()
    dist, normal = torch.empty(P, device=dev), torch.empty(3 * P, device=dev)
    wmax = torch.zeros(vox.n, device=dev)
    r.forward(rgb, depth, alpha, wmax, dist=dist, normal=normal)
    torch.cuda.synchronize()
    say(f"{N_VIEWS} views: auxiliary channels and terms")
    ref = oracle.render_aux(scene, cams)
    for name, got in (("dist", dist), ("normal", normal)):
        e = np.abs(got.cpu().numpy().astype(np.float64) - ref[name]).max()
        say(f"  {name} max abs err {e:.2e}")
        assert e <= IMG_TOL, name
    # the terms on the oracle's channels (rounded to binary32, the kernel's input)
    f64 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    ch = [f64(ref[k]) for k in ("depth", "alpha", "normal", "dist")]
    lam = (0.3, 0.7, 1.9)
    L_ref, ga, gd, gn, gl = oaux.aux_losses(*ch, cams, *lam)
    loss = torch.full((4 * N_VIEWS,), 7.0, device=dev)
    bufs = [torch.full((P,), 9.0, device=dev), torch.full((P,), 9.0, device=dev),
            torch.full((3 * P,), 9.0, device=dev), torch.full((P,), 9.0, device=dev)]
    lv.aux_loss(ctx, frame, *(to_dev(c, dev) for c in ch), *lam, loss, *bufs)
    torch.cuda.synchronize()
    Lg = loss.cpu().numpy().astype(np.float64).reshape(N_VIEWS, 4)
    assert np.allclose(Lg, L_ref, rtol=1e-4, atol=1e-7)
    for name, g, rf in (("alpha", bufs[0], ga), ("depth", bufs[1], gd), ("normal", bufs[2], gn),
                        ("dist", bufs[3], gl)):
        e = rel_l2(g.cpu().numpy().astype(np.float64), rf)
        say(f"  d_{name} rel-L2 {e:.2e}")
        assert e <= 1e-4, name


def test_max_views_loss_weight_l1_and_depth_quantile(ctx, problem):
    import torch
    import paper_2511_02510_amd as lv
    scene, cams = problem
    dev = ctx.device
    rng = np.random.default_rng(154)
    targets = [synth.make_target(rng, c.width, c.height) for c in cams]
    rgbs = [rng.uniform(0, 1, (3, c.height, c.width)).astype(np.float32) for c in cams]
    frame = lv.Frame(cams, dev)
    cat = lambda xs: to_dev(np.concatenate([x.ravel() for x in xs]), dev)
    say(f"{N_VIEWS} views: loss weight, L1 gradient, depth quantile")
    w = torch.empty(frame.P, device=dev)
    ws = torch.empty(lv.lf_weight_workspace_size(N_VIEWS), dtype=torch.uint8, device=dev)
    lv.lf_weight(ctx, frame, cat(targets), 0.5, 1, 1e-3, w, ws)
    torch.cuda.synchronize()
    got = w.cpu().numpy().astype(np.float64)
    wref = [oloss.lf_weight(t, 0.5, 1) for t in targets]
    ref = np.concatenate([x.ravel() for x in wref])
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
    loss = torch.empty(N_VIEWS, device=dev)
    g = torch.empty(3 * frame.P, device=dev)
    lv.l1_grad(ctx, frame, cat(rgbs), cat(targets), cat(wref), loss, g)
    torch.cuda.synchronize()
    lg = loss.cpu().numpy()
    for v in (0, 1, 127, 254, 255):
        l_ref, g_ref = oloss.l1_loss_grad(rgbs[v], targets[v], wref[v])
        assert abs(lg[v] - l_ref) < 1e-5 * max(1.0, abs(l_ref))
        gv = frame.view_rgb(g, v).cpu().numpy()
        assert np.abs(gv - g_ref).max() < 1e-6 * np.abs(g_ref).max() + 1e-12
    # depth quantile: every voxel's proxy is a minimum over all 256 views
    vox = lv.Voxels.from_scene(scene, dev)
    wm = np.round(rng.random(scene.n) ** 2, 3).astype(np.float32)
    qws = torch.empty(lv.quantile_workspace_size(vox.n, 16), dtype=torch.uint8, device=dev)
    tau = torch.empty(16, device=dev)
    prune = torch.empty(vox.n, dtype=torch.uint8, device=dev)
    bins = torch.empty(vox.n, dtype=torch.uint8, device=dev)
    lv.depth_quantile(ctx, vox, frame, to_dev(wm, dev), 16, 0.2, qws, tau, prune, bins)
    torch.cuda.synchronize()
    qref = oquant.depth_quantile(scene, cams, wm, 16, 0.2)
    assert np.array_equal(bins.cpu().numpy(), qref["bins"])
    assert np.array_equal(tau.cpu().numpy(), qref["tau"])
    assert np.array_equal(prune.cpu().numpy(), qref["prune"])


def _strip_camera(o, width, height):
    """A view of the largest side the ABI takes in one direction and a few
    pixels in the other, with square pixels and the usual field of view
    along the long side (a thin strip through the scene)."""
    c = look_at(o, width, height)
    foc = c.fx if width >= height else look_at(o, height, width).fx
    return synth.Camera(R=c.R, o=c.o, fx=foc, fy=foc, cx=width / 2.0, cy=height / 2.0,
                        width=width, height=height)


def test_max_image_sides(ctx):
    # 32767 x 3 and 3 x 32767 pixels (the side limit): pixel coordinates and
    # ranges at the top of their 16-bit fields, rows of 4096 tiles at tile 8
    scene = small_shell(6000, seed=155, deg=1, lmin=4, lmax=7, clutter=0.2)
    cams = [_strip_camera((2.1, 0.63, 1.37), 32767, 3), _strip_camera((-1.4, 0.91, 2.03), 3, 32767),
            look_at((0.7, -2.2, 1.1), 33, 21)]
    P = sum(c.npix for c in cams)
    say("views of 32767 x 3, 3 x 32767 and 33 x 21 px: keys, forward, backward")
    grads = random_grads(np.random.default_rng(156), P)
    ref = oracle.render(scene, cams)
    assert ref["alpha"][:cams[0].npix].max() > 0.1 and ref["alpha"][cams[0].npix:].max() > 0.1
    dd, dsh = oracle.backward(scene, cams, *grads)
    for tile in (8, 32):
        g = run_gpu(ctx, scene, cams, tile=tile, chunk=64, grads=grads)
        check_keys(g["bins"], scene, cams, tile)
        check_images(g, ref)
        assert np.abs(g["wmax"] - ref["wmax"]).max() <= WMAX_TOL
        e1, e2 = rel_l2(g["dd"], dd), rel_l2(g["dsh"], dsh)
        say(f"  tile {tile}: gradient rel-L2 density {e1:.2e} sh {e2:.2e}")
        assert e1 <= GRAD_TOL and e2 <= GRAD_TOL
