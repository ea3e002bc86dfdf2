"""GPU parity of the grid-point density layout and the density activations
(the storage of the sparse-voxel rasterizer the paper starts from): images
and w_max against the FP64 oracle on the gathered corners, gradients with
respect to the stored grid values against the oracle's adjoint scattered
through the activation, the identity layout bit-identical to the dense one,
out-of-range indices reading 0, and argument errors."""
import numpy as np
import pytest

import oracle
from oracle import grid as ogrid
import synth
from synth.scenes import look_at
from gpu_helpers import (GRAD_TOL, IMG_TOL, WMAX_TOL, random_grads, rel_l2, say, small_shell,
                         to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_02510_amd as lv
    c = lv.Context(0)
    yield c
    c.close()


CAMS = [look_at((2.0, 0.7, 1.2), 96, 72), look_at((-0.7, 1.2, -2.0), 80, 60)]


def _run(ctx, vox, cams, grads):
    import paper_2511_02510_amd as lv
    import torch
    dev = ctx.device
    frame = lv.Frame(cams, dev)
    r = lv.Renderer(ctx, vox, frame, lv.settings(tile=16, chunk=64))
    rgb, depth, alpha = r.new_outputs()
    wmax = torch.zeros(vox.n, device=dev)
    r.forward(rgb, depth, alpha, wmax)
    dd = torch.empty_like(vox.density)
    dsh = torch.empty_like(vox.sh)
    r.backward(to_dev(grads[0], dev), to_dev(grads[1], dev), to_dev(grads[2], dev), dd, dsh)
    torch.cuda.synchronize()
    f = lambda t: t.cpu().numpy().astype(np.float64)
    return dict(rgb=f(rgb), depth=f(depth), alpha=f(alpha), wmax=f(wmax), dd=f(dd), dsh=f(dsh))


def _check(g, ref, dd_ref, dsh_ref):
    for k in ("rgb", "depth", "alpha"):
        assert np.abs(g[k] - ref[k]).max() <= IMG_TOL, k
    assert np.abs(g["wmax"] - ref["wmax"]).max() <= WMAX_TOL
    e1, e2 = rel_l2(g["dd"], dd_ref), rel_l2(g["dsh"], dsh_ref)
    say(f"  rel L2: density {e1:.2e} sh {e2:.2e}")
    assert e1 <= GRAD_TOL and e2 <= GRAD_TOL


@pytest.mark.parametrize("act", [ogrid.ACT_NONE, ogrid.ACT_SOFTPLUS, ogrid.ACT_EXP])
def test_grid_layout_forward_and_gradient(ctx, act):
    import paper_2511_02510_amd as lv
    scene = small_shell(20000, seed=51 + act, deg=1, lmin=5, lmax=9, clutter=0.1)
    idx, ng = synth.grid_points(scene)
    rng = np.random.default_rng(52 + act)
    # stored values drawn so that the corner densities span the range of the
    # other workloads (softplus of N(0, 2): mostly below 8)
    if act == ogrid.ACT_NONE:
        raw = np.abs(rng.normal(1.0, 1.0, ng))
    elif act == ogrid.ACT_SOFTPLUS:
        raw = rng.normal(0.0, 1.0, ng)
    else:
        raw = rng.normal(-0.5, 0.6, ng)
    raw = raw.astype(np.float32)
    say(f"grid layout, act {act}: {scene.n} voxels on {ng} points")
    P = sum(c.npix for c in CAMS)
    grads = random_grads(rng, P)
    vox = lv.Voxels.from_grid(scene, idx, raw, ctx.device, act=act)
    g = _run(ctx, vox, CAMS, grads)
    dense = ogrid.with_corners(scene, ogrid.corner_values(raw, idx, act))
    ref = oracle.render(dense, CAMS)
    dc, dsh = oracle.backward(dense, CAMS, *grads)
    _check(g, ref, ogrid.grid_gradient(dc, raw, idx, act), dsh)
    assert g["dd"].shape == (ng,)


@pytest.mark.parametrize("act", [ogrid.ACT_SOFTPLUS, ogrid.ACT_EXP])
def test_dense_layout_with_activation(ctx, act):
    import paper_2511_02510_amd as lv
    scene = small_shell(20000, seed=61, deg=2, lmin=5, lmax=9)
    rng = np.random.default_rng(62)
    scene.density = rng.normal(-0.5, 1.0, scene.density.shape).astype(np.float32)
    say(f"dense layout, act {act}")
    grads = random_grads(rng, sum(c.npix for c in CAMS))
    g = _run(ctx, lv.Voxels.from_scene(scene, ctx.device, act=act), CAMS, grads)
    raw = scene.density.astype(np.float64)
    dense = ogrid.with_corners(scene, ogrid.activate(raw, act))
    ref = oracle.render(dense, CAMS)
    dc, dsh = oracle.backward(dense, CAMS, *grads)
    _check(g, ref, dc * ogrid.activate_grad(raw, act), dsh)


def test_identity_grid_layout_is_the_dense_layout(ctx):
    import paper_2511_02510_amd as lv
    scene = small_shell(15000, seed=71, deg=1, lmin=5, lmax=9)
    n = scene.n
    idx = (np.arange(8)[:, None] * n + np.arange(n)[None, :]).astype(np.int32)
    rng = np.random.default_rng(72)
    grads = random_grads(rng, sum(c.npix for c in CAMS))
    say("identity grid layout vs dense layout")
    a = _run(ctx, lv.Voxels.from_scene(scene, ctx.device), CAMS, grads)
    b = _run(ctx, lv.Voxels.from_grid(scene, idx, scene.density.ravel(), ctx.device), CAMS, grads)
    for k in ("rgb", "depth", "alpha", "wmax"):
        assert np.array_equal(a[k], b[k]), k
    assert rel_l2(b["dd"], a["dd"].ravel()) <= 1e-6
    assert rel_l2(b["dsh"], a["dsh"]) <= 1e-6


def test_out_of_range_indices_read_zero(ctx):
    import paper_2511_02510_amd as lv
    scene = small_shell(10000, seed=81, deg=0, lmin=5, lmax=8)
    idx, ng = synth.grid_points(scene)
    rng = np.random.default_rng(82)
    bad = rng.choice(idx.size, 500, replace=False)
    idx.ravel()[bad[:250]] = -3
    idx.ravel()[bad[250:]] = ng + 17
    raw = rng.normal(0.0, 1.0, ng).astype(np.float32)
    grads = random_grads(rng, sum(c.npix for c in CAMS))
    say("grid indices out of range")
    g = _run(ctx, lv.Voxels.from_grid(scene, idx, raw, ctx.device, act=ogrid.ACT_SOFTPLUS), CAMS, grads)
    dense = ogrid.with_corners(scene, ogrid.corner_values(raw, idx, ogrid.ACT_SOFTPLUS))
    assert np.count_nonzero(dense.density == 0.0) == 500
    ref = oracle.render(dense, CAMS)
    dc, dsh = oracle.backward(dense, CAMS, *grads)
    _check(g, ref, ogrid.grid_gradient(dc, raw, idx, ogrid.ACT_SOFTPLUS), dsh)


def test_autograd_through_the_grid_layout(ctx):
    import paper_2511_02510_amd as lv
    import torch
    scene = small_shell(8000, seed=95, deg=1, lmin=5, lmax=8)
    idx, ng = synth.grid_points(scene)
    rng = np.random.default_rng(96)
    raw = rng.normal(0.0, 1.0, ng).astype(np.float32)
    vox = lv.Voxels.from_grid(scene, idx, raw, ctx.device, act=ogrid.ACT_SOFTPLUS)
    frame = lv.Frame(CAMS, ctx.device)
    r = lv.Renderer(ctx, vox, frame, lv.settings())
    P = frame.P
    g_rgb = to_dev(rng.normal(0, 1e-3, 3 * P), ctx.device)
    g_alpha = to_dev(rng.normal(0, 1e-3, P), ctx.device)
    say("autograd through the grid layout")
    density = vox.density.clone().requires_grad_(True)
    sh = vox.sh.clone().requires_grad_(True)
    wmax = torch.zeros(vox.n, device=ctx.device)
    rgb, depth, alpha = lv.rasterize(density, sh, r, wmax)
    ((rgb * g_rgb).sum() + (alpha * g_alpha).sum()).backward()
    dd = torch.empty_like(vox.density)
    dsh = torch.empty_like(vox.sh)
    r.forward(*r.new_outputs(), torch.zeros(vox.n, device=ctx.device))
    r.backward(g_rgb, None, g_alpha, dd, dsh)
    torch.cuda.synchronize()
    assert density.grad.shape == (ng,)
    assert rel_l2(density.grad.cpu().numpy(), dd.cpu().numpy()) <= 1e-5
    assert rel_l2(sh.grad.cpu().numpy(), dsh.cpu().numpy()) <= 1e-5


def test_grid_layout_argument_errors(ctx):
    import paper_2511_02510_amd as lv
    import torch
    scene = small_shell(3000, seed=91, deg=0, lmin=4, lmax=7)
    idx, ng = synth.grid_points(scene)
    vox = lv.Voxels.from_grid(scene, idx, np.zeros(ng, np.float32), ctx.device)
    frame = lv.Frame(CAMS[:1], ctx.device)
    say("grid layout argument errors")
    vox.struct.density_act = 7
    with pytest.raises(lv.LiteVoxelError):
        lv.query_sizes(ctx, vox, frame, lv.settings())
    vox.struct.density_act = 0
    split = torch.zeros(vox.n, dtype=torch.uint8, device=ctx.device)
    ws = torch.empty(lv.split_workspace_size(vox.n), dtype=torch.uint8, device=ctx.device)
    with pytest.raises(lv.LiteVoxelError):
        lv.subdivide_apply(ctx, vox, split, vox.n, ws)
