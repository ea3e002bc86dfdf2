"""GPU parity of the auxiliary render channels and terms (eq. 6 and 17 name
them; readings in include/litevoxel.h and oracle/): the distortion, normal and
median-depth channels of lv_forward_aux, the adjoint of lv_backward_aux, the
image terms of lv_aux_loss, and the whole chain channels -> terms -> gradient,
against the FP64 oracle on the same seeded inputs, through the C-ABI.

The median depth is the chord midpoint of the hit at which the transmittance
first reaches 1/2: where the oracle's transmittance after some hit lies
within 1e-4 of 1/2, binary32 may cross at the neighbouring hit, so the GPU
value must equal the oracle's median depth at one of the thresholds
1/2 - 1e-4 and 1/2 + 1e-4 (equal wherever the crossing is clear)."""
import numpy as np
import pytest

import oracle
from oracle import aux as oaux
from synth.scenes import look_at
from gpu_helpers import GRAD_TOL, IMG_TOL, WMAX_TOL, check_images, rel_l2, say, small_shell, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_02510_amd as lv
    c = lv.Context(0)
    yield c
    c.close()


def _scene():
    sc = small_shell(20000, seed=81, deg=2, lmin=4, lmax=9, clutter=0.1)
    cams = [look_at((2.0, 0.7, 1.3), 96, 72), look_at((-1.3, 0.6, -2.1), 80, 60),
            look_at((0.4, -2.2, 1.1), 67, 53)]
    return sc, cams


def _render(ctx, sc, cams, tile=16, chunk=64, chunk_bwd=0, vox=None, bg=(0.0, 0.0, 0.0)):
    import torch
    import paper_2511_02510_amd as lv
    dev = ctx.device
    vox = lv.Voxels.from_scene(sc, dev) if vox is None else vox
    frame = lv.Frame(cams, dev, bg=bg)
    r = lv.Renderer(ctx, vox, frame, lv.settings(tile=tile, chunk=chunk, chunk_bwd=chunk_bwd))
    rgb, depth, alpha = r.new_outputs()
    P = frame.P
    dist, normal = torch.empty(P, device=dev), torch.empty(3 * P, device=dev)
    mdepth = torch.empty(P, device=dev)
    wmax = torch.zeros(vox.n, device=dev)
    r.forward(rgb, depth, alpha, wmax, dist=dist, normal=normal, mdepth=mdepth)
    torch.cuda.synchronize()
    return r, vox, frame, dict(rgb=rgb, depth=depth, alpha=alpha, dist=dist, normal=normal,
                               wmax=wmax, mdepth=mdepth)


def check_mdepth(got, scene, cams):
    """The GPU median depth against the oracle's crossing band; returns the
    number of pixels whose crossing lies in the band."""
    lo = oracle.median_depth(scene, cams, 0.5 + 1e-4)
    hi = oracle.median_depth(scene, cams, 0.5 - 1e-4)
    ok = (np.abs(got - lo) <= IMG_TOL) | (np.abs(got - hi) <= IMG_TOL)
    amb = int(np.count_nonzero(lo != hi))
    say(f"  median depth: {int(np.count_nonzero(hi))} px with a crossing, {amb} in the band, "
        f"{int(np.count_nonzero(~ok))} off")
    assert ok.all()
    assert amb <= 1e-3 * got.size + 2
    return amb


def _np(t):
    return t.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("tile,chunk", [(16, 64), (8, 256), (32, 128)])
def test_aux_channels_forward(ctx, tile, chunk):
    import torch
    sc, cams = _scene()
    say(f"aux forward: {sc.n} voxels, 3 views, tile {tile} chunk {chunk}")
    r, vox, frame, out = _render(ctx, sc, cams, tile, chunk)
    ref = oracle.render_aux(sc, cams)
    got = {k: _np(v) for k, v in out.items()}
    check_images(got, ref)
    check_mdepth(got["mdepth"], sc, cams)
    assert np.count_nonzero(got["mdepth"]) > 300   # pixels where the opacity reaches 1/2
    e_w = float(np.abs(got["wmax"] - ref["wmax"]).max())
    e_l = float(np.abs(got["dist"] - ref["dist"]).max())
    e_n = float(np.abs(got["normal"] - ref["normal"]).max())
    say(f"  w_max {e_w:.2e}  dist {e_l:.2e} (max {ref['dist'].max():.3e})  normal {e_n:.2e}")
    assert e_w <= WMAX_TOL and e_l <= IMG_TOL and e_n <= IMG_TOL
    assert ref["dist"].max() > 1e-3 and np.abs(ref["normal"]).max() > 0.3
    # the plain channels are the plain forward's, bit for bit
    rgb, depth, alpha = r.new_outputs()
    wm = torch.zeros(vox.n, device=ctx.device)
    r.forward(rgb, depth, alpha, wm)
    torch.cuda.synchronize()
    for k, t in (("rgb", rgb), ("depth", depth), ("alpha", alpha), ("wmax", wm)):
        assert torch.equal(t, out[k]), k


@pytest.mark.parametrize("which,tile,chunk", [("all", 16, 64), ("dist", 16, 64),
                                              ("normal", 16, 64), ("all", 8, 256),
                                              ("all", 32, 128)])
def test_aux_backward_matches_oracle(ctx, which, tile, chunk):
    import torch
    sc, cams = _scene()
    r, vox, frame, out = _render(ctx, sc, cams, tile, chunk)
    P = frame.P
    rng = np.random.default_rng(82)
    g_rgb = rng.normal(0, 1e-3, 3 * P)
    g_depth = rng.normal(0, 1e-4, P)
    g_alpha = rng.normal(0, 1e-3, P)
    g_dist = rng.normal(0, 1e-2, P) if which in ("all", "dist") else None
    g_normal = rng.normal(0, 1e-3, 3 * P) if which in ("all", "normal") else None
    dev = ctx.device
    dd, dsh = torch.empty_like(vox.density), torch.empty_like(vox.sh)
    t = lambda a: None if a is None else to_dev(a, dev)
    r.backward_aux(t(g_rgb), t(g_depth), t(g_alpha), out["depth"], t(g_dist), t(g_normal), dd, dsh)
    torch.cuda.synchronize()
    dd_ref, dsh_ref = oracle.backward_aux(sc, cams, g_rgb, g_depth, g_alpha, g_dist, g_normal)
    e = rel_l2(np.concatenate([_np(dd).ravel(), _np(dsh).ravel()]),
               np.concatenate([dd_ref.ravel(), dsh_ref.ravel()]))
    # the auxiliary part alone
    dd0, dsh0 = oracle.backward(sc, cams, g_rgb, g_depth, g_alpha)
    e_aux = rel_l2(_np(dd) - dd0, dd_ref - dd0)
    say(f"  aux backward [{which}, tile {tile} chunk {chunk}]: gradient rel-L2 {e:.2e}, "
        f"density part of the aux terms {e_aux:.2e}")
    assert e <= GRAD_TOL and e_aux <= GRAD_TOL


def test_aux_loss_kernel_matches_oracle(ctx):
    import torch
    import paper_2511_02510_amd as lv
    # ragged tiles, a view without interior pixels, and a view of more tiles
    # (11 x 33) than the kernel launches blocks per view
    cams = [look_at((0.3, 0.4, -2.5), 64, 48), look_at((2.0, 0.1, 0.5), 37, 29),
            look_at((1.0, 1.0, 1.0), 2, 9), look_at((-1.5, 0.7, 2.0), 331, 259)]
    frame = lv.Frame(cams, ctx.device)
    P = frame.P
    rng = np.random.default_rng(83)
    depth = np.concatenate([
        (2.5 + 0.3 * np.sin(np.arange(c.npix) * 0.01) + rng.normal(0, 0.01, c.npix)) for c in cams])
    alpha = rng.uniform(0, 1, P)
    normal = rng.normal(0, 0.4, 3 * P)
    dist = rng.uniform(0, 0.05, P)
    lam = (0.3, 0.7, 1.9)
    # a median-depth map: the depth with a bump (a different surface), zeros
    # where no hit reached one half
    mdepth = depth + 0.05 * np.cos(np.arange(P) * 0.003)
    mdepth[rng.random(P) < 0.05] = 0.0
    depth, alpha, normal, dist, mdepth = (np.asarray(x, np.float32).astype(np.float64)
                                          for x in (depth, alpha, normal, dist, mdepth))
    L_ref, ga, gd, gn, gl = oaux.aux_losses(depth, alpha, normal, dist, cams, *lam, mdepth=mdepth,
                                            lam_nm=1.1)
    dev = ctx.device
    f32 = lambda a: to_dev(a, dev)
    loss = torch.full((4 * len(cams),), 7.0, device=dev)
    bufs = [torch.full((P,), 9.0, device=dev), torch.full((P,), 9.0, device=dev),
            torch.full((3 * P,), 9.0, device=dev), torch.full((P,), 9.0, device=dev)]
    lv.aux_loss(ctx, frame, f32(depth), f32(alpha), f32(normal), f32(dist), *lam, loss, *bufs,
                mdepth=f32(mdepth), lam_nm=1.1)
    torch.cuda.synchronize()
    Lg = _np(loss).reshape(len(cams), 4)
    say(f"  aux losses GPU {Lg.ravel()} oracle {L_ref.ravel()}")
    assert np.allclose(Lg, L_ref, rtol=1e-4, atol=1e-7)
    for name, g, ref in (("alpha", bufs[0], ga), ("depth", bufs[1], gd), ("normal", bufs[2], gn),
                         ("dist", bufs[3], gl)):
        e = rel_l2(_np(g), ref)
        say(f"  d_{name} rel-L2 {e:.2e}")
        assert e <= 1e-4, name


def test_aux_chain_loss_and_gradient(ctx):
    """channels -> image terms -> gradient, the whole chain on both sides."""
    import torch
    import paper_2511_02510_amd as lv
    sc, cams = _scene()
    r, vox, frame, out = _render(ctx, sc, cams, 16, 64)
    lam = (0.05, 0.2, 5.0)
    dev, P = ctx.device, frame.P
    loss = torch.empty(4 * len(cams), device=dev)
    ga, gd, gl = (torch.empty(P, device=dev) for _ in range(3))
    gn = torch.empty(3 * P, device=dev)
    lv.aux_loss(ctx, frame, out["depth"], out["alpha"], out["normal"], out["dist"], *lam, loss, ga,
                gd, gn, gl, mdepth=out["mdepth"], lam_nm=0.3)
    dd, dsh = torch.empty_like(vox.density), torch.empty_like(vox.sh)
    zero_rgb = torch.zeros(3 * P, device=dev)
    r.backward_aux(zero_rgb, gd, ga, out["depth"], gl, gn, dd, dsh)
    torch.cuda.synchronize()
    ref = oracle.render_aux(sc, cams)
    L_ref, ga_r, gd_r, gn_r, gl_r = oaux.aux_losses(ref["depth"], ref["alpha"], ref["normal"],
                                                    ref["dist"], cams, *lam,
                                                    mdepth=oracle.median_depth(sc, cams),
                                                    lam_nm=0.3)
    dd_r, dsh_r = oracle.backward_aux(sc, cams, np.zeros(3 * P), gd_r, ga_r, gl_r, gn_r)
    Lg = _np(loss).reshape(len(cams), 4)
    say(f"  chain losses GPU {Lg.ravel()} oracle {L_ref.ravel()}")
    assert np.allclose(Lg, L_ref, rtol=1e-3, atol=1e-6)
    e = rel_l2(_np(dd), dd_r)
    say(f"  chain gradient rel-L2 {e:.2e}")
    assert e <= GRAD_TOL
    assert np.all(_np(dsh) == 0.0)    # no colour term in this loss


def test_aux_autograd_matches_direct_calls(ctx):
    import torch
    import paper_2511_02510_amd as lv
    sc, cams = _scene()
    dev = ctx.device
    vox = lv.Voxels.from_scene(sc, dev)
    frame = lv.Frame(cams, dev)
    r = lv.Renderer(ctx, vox, frame, lv.settings(tile=16, chunk=64))
    dens = vox.density.clone().requires_grad_(True)
    sh = vox.sh.clone().requires_grad_(True)
    wmax = torch.zeros(vox.n, device=dev)
    rgb, depth, alpha, dist, normal, mdepth = lv.rasterize_aux(dens, sh, r, wmax)
    assert not mdepth.requires_grad
    rng = np.random.default_rng(84)
    P = frame.P
    w = [to_dev(rng.normal(0, s, n), dev) for s, n in ((1e-3, 3 * P), (1e-4, P), (1e-3, P),
                                                       (1e-2, P), (1e-3, 3 * P))]
    L = sum((o * wi).sum() for o, wi in zip((rgb, depth, alpha, dist, normal), w))
    L.backward()
    torch.cuda.synchronize()
    dd_ref, dsh_ref = oracle.backward_aux(sc, cams, *[_np(x) for x in w])
    e = rel_l2(np.concatenate([_np(dens.grad).ravel(), _np(sh.grad).ravel()]),
               np.concatenate([dd_ref.ravel(), dsh_ref.ravel()]))
    say(f"  autograd aux gradient rel-L2 {e:.2e}")
    assert e <= GRAD_TOL


def _aux_grads(rng, P):
    return (rng.normal(0, 1e-3, 3 * P), rng.normal(0, 1e-4, P), rng.normal(0, 1e-3, P),
            rng.normal(0, 1e-2, P), rng.normal(0, 1e-3, 3 * P))


def _aux_case(ctx, sc, cams, grads, ref_scene, tile, chunk, vox=None, bg=(0.0, 0.0, 0.0)):
    """Forward channels and the full auxiliary gradient of one case, both
    sides; returns the GPU gradients and the oracle's corner gradient."""
    import torch
    r, vox, frame, out = _render(ctx, sc, cams, tile, chunk, vox=vox, bg=bg)
    ref = oracle.render_aux(ref_scene, cams, bg=bg)
    got = {k: _np(v) for k, v in out.items()}
    check_images(got, ref)
    e_l = float(np.abs(got["dist"] - ref["dist"]).max())
    e_n = float(np.abs(got["normal"] - ref["normal"]).max())
    say(f"  dist {e_l:.2e} (max {ref['dist'].max():.3e})  normal {e_n:.2e}")
    assert float(np.abs(got["wmax"] - ref["wmax"]).max()) <= WMAX_TOL
    assert e_l <= IMG_TOL and e_n <= IMG_TOL
    dev = ctx.device
    dd, dsh = torch.empty_like(vox.density), torch.empty_like(vox.sh)
    g = [to_dev(a, dev) for a in grads]
    r.backward_aux(g[0], g[1], g[2], out["depth"], g[3], g[4], dd, dsh)
    torch.cuda.synchronize()
    dd_ref, dsh_ref = oracle.backward_aux(ref_scene, cams, *grads, bg=bg)
    return _np(dd), _np(dsh), dd_ref, dsh_ref


def test_aux_camera_inside_scene(ctx):
    """The near plane cuts voxels around the camera; chords start at t = 0."""
    sc = small_shell(5000, seed=85, deg=1, lmin=4, lmax=7, clutter=0.5)
    cams = [look_at((0.05, 0.02, 0.79), 50, 40, target=(0.3, 0.1, -0.5)),
            look_at((-0.1, 0.3, 0.2), 41, 37, target=(0.5, -0.6, 0.1))]
    say("aux channels, camera inside the root cube")
    grads = _aux_grads(np.random.default_rng(86), sum(c.npix for c in cams))
    dd, dsh, dd_ref, dsh_ref = _aux_case(ctx, sc, cams, grads, sc, 8, 64)
    e1, e2 = rel_l2(dd, dd_ref), rel_l2(dsh, dsh_ref)
    say(f"  gradient rel-L2 density {e1:.2e} sh {e2:.2e}")
    assert e1 <= GRAD_TOL and e2 <= GRAD_TOL


def test_aux_with_background(ctx):
    """The background enters the colour only: the normal channel carries no
    background term and the distortion none either."""
    sc, cams = _scene()
    bg = (0.2, 0.5, 0.9)
    say(f"aux channels, background {bg}")
    grads = _aux_grads(np.random.default_rng(87), sum(c.npix for c in cams))
    dd, dsh, dd_ref, dsh_ref = _aux_case(ctx, sc, cams, grads, sc, 16, 128, bg=bg)
    e1, e2 = rel_l2(dd, dd_ref), rel_l2(dsh, dsh_ref)
    say(f"  gradient rel-L2 density {e1:.2e} sh {e2:.2e}")
    assert e1 <= GRAD_TOL and e2 <= GRAD_TOL


def test_aux_grid_layout_softplus(ctx):
    """Grid-point storage through softplus: the voxel normal and its
    Jacobian act on the activated corner values, and the corner gradient is
    scattered onto the stored grid values."""
    import paper_2511_02510_amd as lv
    import synth
    from oracle import grid as ogrid
    sc = small_shell(20000, seed=88, deg=1, lmin=5, lmax=9, clutter=0.1)
    idx, ng = synth.grid_points(sc)
    rng = np.random.default_rng(89)
    raw = rng.normal(0.0, 1.0, ng).astype(np.float32)
    cams = [look_at((2.0, 0.7, 1.2), 96, 72), look_at((-0.7, 1.2, -2.0), 80, 60)]
    say(f"aux channels, grid layout through softplus: {sc.n} voxels on {ng} points")
    vox = lv.Voxels.from_grid(sc, idx, raw, ctx.device, act=ogrid.ACT_SOFTPLUS)
    dense = ogrid.with_corners(sc, ogrid.corner_values(raw, idx, ogrid.ACT_SOFTPLUS))
    grads = _aux_grads(rng, sum(c.npix for c in cams))
    dd, dsh, dc_ref, dsh_ref = _aux_case(ctx, sc, cams, grads, dense, 16, 64, vox=vox)
    dd_ref = ogrid.grid_gradient(dc_ref, raw, idx, ogrid.ACT_SOFTPLUS)
    assert dd.shape == (ng,)
    e1, e2 = rel_l2(dd, dd_ref), rel_l2(dsh, dsh_ref)
    say(f"  gradient rel-L2 grid values {e1:.2e} sh {e2:.2e}")
    assert e1 <= GRAD_TOL and e2 <= GRAD_TOL


def test_aux_forward_with_one_channel(ctx):
    """Either channel may be omitted: the other one and the plain outputs are
    those of the call with both."""
    import torch
    sc, cams = _scene()
    r, vox, frame, out = _render(ctx, sc, cams, 16, 64)
    P = frame.P
    for keep in ("dist", "normal", "mdepth"):
        rgb, depth, alpha = r.new_outputs()
        wm = torch.zeros(vox.n, device=ctx.device)
        ch = {k: (torch.full(((3 if k == "normal" else 1) * P,), 7.0, device=ctx.device)
                  if k == keep else None) for k in ("dist", "normal", "mdepth")}
        r.forward(rgb, depth, alpha, wm, **ch)
        torch.cuda.synchronize()
        got = ch[keep]
        assert torch.equal(got, out[keep]), keep
        for k, t in (("rgb", rgb), ("depth", depth), ("alpha", alpha), ("wmax", wm)):
            assert torch.equal(t, out[k]), (keep, k)


def test_aux_channels_of_an_empty_scene(ctx):
    """No voxel in front of the camera: both channels are 0 and the
    backward gives zero gradients."""
    import torch
    import paper_2511_02510_amd as lv
    sc, _ = _scene()
    cams = [look_at((0.0, 0.0, 3.0), 40, 30, target=(0.0, 0.0, 9.0))]   # looking away
    r, vox, frame, out = _render(ctx, sc, cams, 16, 64)
    assert float(out["dist"].abs().max()) == 0.0 and float(out["normal"].abs().max()) == 0.0
    assert float(out["alpha"].abs().max()) == 0.0
    P = frame.P
    dd, dsh = torch.empty_like(vox.density), torch.empty_like(vox.sh)
    ones = lambda n: torch.ones(n, device=ctx.device)
    r.backward_aux(ones(3 * P), ones(P), ones(P), out["depth"], ones(P), ones(3 * P), dd, dsh)
    torch.cuda.synchronize()
    assert float(dd.abs().max()) == 0.0 and float(dsh.abs().max()) == 0.0


def test_aux_argument_errors(ctx):
    import torch
    import paper_2511_02510_amd as lv
    sc, cams = _scene()
    r, vox, frame, out = _render(ctx, sc, cams, 16, 64)
    P = frame.P
    dd, dsh = torch.empty_like(vox.density), torch.empty_like(vox.sh)
    g = torch.zeros(P, device=ctx.device)
    with pytest.raises(lv.LiteVoxelError):   # d_dist without the forward's depth
        r.backward_aux(torch.zeros(3 * P, device=ctx.device), None, None, None, g, None, dd, dsh)
    loss = torch.empty(4 * frame.n_views, device=ctx.device)
    bufs = [torch.empty(P, device=ctx.device), torch.empty(P, device=ctx.device),
            torch.empty(3 * P, device=ctx.device), torch.empty(P, device=ctx.device)]
    with pytest.raises(lv.LiteVoxelError):   # every gradient buffer of lv_aux_loss is required
        lv.aux_loss(ctx, frame, out["depth"], out["alpha"], out["normal"], out["dist"], 1.0, 1.0,
                    1.0, loss, bufs[0], None, bufs[2], bufs[3])
    with pytest.raises(lv.LiteVoxelError):   # the median term needs the median depth
        lv.aux_loss(ctx, frame, out["depth"], out["alpha"], out["normal"], out["dist"], 1.0, 1.0,
                    1.0, loss, *bufs, lam_nm=1.0)


def test_aux_step_graph_replays_match_eager(ctx):
    """forward with both channels, the three terms and the backward with
    every channel's gradient, captured once: replays (with eager work between
    them) equal the eager step; the channels bit for bit, the summed losses
    and the gradients up to the order of their atomic sums."""
    import torch
    import paper_2511_02510_amd as lv
    sc, cams = _scene()
    dev = ctx.device
    vox = lv.Voxels.from_scene(sc, dev)
    frame = lv.Frame(cams, dev)
    r = lv.Renderer(ctx, vox, frame, lv.settings(tile=16, chunk=128, chunk_bwd=64))
    P, V = frame.P, frame.n_views
    rgb, depth, alpha = r.new_outputs()
    dist, normal = torch.empty(P, device=dev), torch.empty(3 * P, device=dev)
    wmax = torch.zeros(vox.n, device=dev)
    loss = torch.empty(4 * V, device=dev)
    ga, gd, gl = (torch.empty(P, device=dev) for _ in range(3))
    gn = torch.empty(3 * P, device=dev)
    d_rgb = to_dev(np.random.default_rng(90).normal(0, 1e-3, 3 * P), dev)
    dd, dsh = torch.empty_like(vox.density), torch.empty_like(vox.sh)
    stream = torch.cuda.Stream()

    def step():
        wmax.zero_()
        r.forward(rgb, depth, alpha, wmax, stream=stream, verify=False, dist=dist, normal=normal)
        lv.aux_loss(ctx, frame, depth, alpha, normal, dist, 0.05, 0.2, 5.0, loss, ga, gd, gn, gl,
                    stream=stream)
        r.backward_aux(d_rgb, gd, ga, depth, gl, gn, dd, dsh, stream=stream)

    def snap():
        torch.cuda.synchronize()
        return [x.clone() for x in (rgb, depth, alpha, dist, normal, wmax, ga, gd, gn, gl, loss,
                                    dd, dsh)]

    say("auxiliary step: graph capture and replays")
    with torch.cuda.stream(stream):
        r.forward(rgb, depth, alpha, wmax, stream=stream, verify=True)   # sizes the capacity
        step()
    eager = snap()
    with torch.cuda.stream(stream):
        lv.graph_begin(ctx, stream)
        step()
        lv.graph_end(ctx, stream)
    try:
        for rep in range(3):
            for x in (rgb, dist, normal, gd, dd):
                x.fill_(-7.0)
            torch.cuda.synchronize()
            lv.graph_launch(ctx, stream)
            got = snap()
            for a, b in zip(got[:10], eager[:10]):      # channels, w_max, image gradients
                assert torch.equal(a, b), f"replay {rep}"
            assert torch.allclose(got[10], eager[10], rtol=1e-5, atol=1e-9), f"replay {rep}"
            for a, b in zip(got[11:], eager[11:]):
                assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) < 1e-5, f"replay {rep}"
            _ = (torch.randn(1000, device=dev) * 2).sum().item()     # eager work between replays
    finally:
        lv.graph_reset(ctx)
