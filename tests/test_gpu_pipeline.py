"""GPU parity of the loss (eq. 7-10) and depth-quantile (eq. 11-12, 14) entry
points, and of the execution structure: autograd wrapper, graph capture and
replay, autotuner."""
import numpy as np
import pytest

import oracle
from oracle import loss as oloss, quantile as oquant
import synth
from synth.scenes import look_at
from gpu_helpers import (GRAD_TOL, IMG_TOL, WMAX_TOL, random_grads, rel_l2, run_gpu, say,
                         small_shell, to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_02510_amd as lv
    c = lv.Context(0)
    yield c
    c.close()


def _ragged_cams():
    return [look_at((2.0, 0.6, 1.3), 77, 53), look_at((-1.5, 1.0, 2.0), 128, 96),
            look_at((0.2, 2.3, -1.1), 31, 64)]


@pytest.mark.parametrize("form,gamma", [(0, 0.6), (1, 0.5), (1, 1.0), (0, 0.0)])
def test_lf_weight_matches_oracle(ctx, form, gamma):
    import paper_2511_02510_amd as lv
    import torch
    cams = _ragged_cams()
    rng = np.random.default_rng(20)
    targets = [synth.make_target(rng, c.width, c.height) for c in cams]
    say(f"lf_weight form={form} gamma={gamma}")
    frame = lv.Frame(cams, ctx.device)
    tgt = to_dev(np.concatenate([t.ravel() for t in targets]), ctx.device)
    w = torch.empty(frame.P, device=ctx.device)
    ws = torch.empty(lv.lf_weight_workspace_size(frame.n_views), dtype=torch.uint8, device=ctx.device)
    lv.lf_weight(ctx, frame, tgt, gamma, form, 1e-3, w, ws)
    got = w.cpu().numpy().astype(np.float64)
    ref = np.concatenate([oloss.lf_weight(t, gamma, form).ravel() for t in targets])
    e = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"  max rel err {e:.2e}")
    assert e < 1e-5
    for v in range(3):
        assert abs(got[frame.off[v]:frame.off[v + 1]].mean() - 1.0) < 1e-5


def test_l1_grad_matches_oracle(ctx):
    import paper_2511_02510_amd as lv
    import torch
    cams = _ragged_cams()
    rng = np.random.default_rng(21)
    targets = [synth.make_target(rng, c.width, c.height) for c in cams]
    rgbs = [rng.uniform(0, 1, (3, c.height, c.width)).astype(np.float32) for c in cams]
    rgbs[0][:, :5, :5] = targets[0][:, :5, :5]          # exact zeros of the residual
    weights = [oloss.lf_weight(t, 0.5, 1) for t in targets]
    say("l1_grad ragged views")
    frame = lv.Frame(cams, ctx.device)
    cat = lambda xs: to_dev(np.concatenate([x.ravel() for x in xs]), ctx.device)
    loss = torch.empty(3, device=ctx.device)
    g = torch.empty(3 * frame.P, device=ctx.device)
    lv.l1_grad(ctx, frame, cat(rgbs), cat(targets), cat(weights), loss, g)
    torch.cuda.synchronize()
    for v in range(3):
        l_ref, g_ref = oloss.l1_loss_grad(rgbs[v], targets[v], weights[v])
        assert abs(loss[v].item() - l_ref) < 1e-5 * max(1.0, abs(l_ref))
        got = frame.view_rgb(g, v).cpu().numpy()
        assert np.abs(got - g_ref).max() < 1e-6 * np.abs(g_ref).max() + 1e-12
    assert np.all(frame.view_rgb(g, 0).cpu().numpy()[:, :5, :5] == 0.0)   # sign(0) = 0


def test_depth_quantile_bit_exact_on_same_wmax(ctx):
    import paper_2511_02510_amd as lv
    import torch
    scene = small_shell(40000, seed=22, lmin=5, lmax=9, clutter=0.1)
    cams = synth.make_cameras_ring(np.random.default_rng(1), 4)
    cams = [look_at(c.o, c.width // 8, c.height // 8) for c in cams]
    say("depth quantile, 40k voxels, 4 views")
    g = run_gpu(ctx, scene, cams, export=False)
    vox = lv.Voxels.from_scene(scene, ctx.device)
    frame = lv.Frame(cams, ctx.device)
    wmax = to_dev(g["wmax"], ctx.device)
    ws = torch.empty(lv.quantile_workspace_size(vox.n, 16), dtype=torch.uint8, device=ctx.device)
    tau = torch.empty(16, device=ctx.device)
    prune = torch.empty(vox.n, dtype=torch.uint8, device=ctx.device)
    bins = torch.empty(vox.n, dtype=torch.uint8, device=ctx.device)
    lv.depth_quantile(ctx, vox, frame, wmax, 16, 0.1, ws, tau, prune, bins)
    torch.cuda.synchronize()
    ref = oquant.depth_quantile(scene, cams, g["wmax"].astype(np.float32), 16, 0.1)
    assert np.array_equal(bins.cpu().numpy(), ref["bins"])
    assert np.array_equal(tau.cpu().numpy(), ref["tau"])
    assert np.array_equal(prune.cpu().numpy(), ref["prune"])
    # against the oracle's own w_max: tau within the w_max tolerance
    ref2 = oquant.depth_quantile(scene, cams, oracle.render(scene, cams)["wmax"], 16, 0.1)
    t_gpu, t_ref = tau.cpu().numpy(), ref2["tau"]
    fin = np.isfinite(t_ref)
    assert np.array_equal(np.isfinite(t_gpu), fin)
    assert np.abs(t_gpu[fin] - t_ref[fin]).max() <= WMAX_TOL
    near = np.abs(g["wmax"] - t_ref[ref2["bins"]]) <= WMAX_TOL
    assert np.all((prune.cpu().numpy() == ref2["prune"]) | near)


def test_depth_bins_then_cutoff_twice(ctx):
    # the split form: the binning once (before any w_max exists), then the
    # cutoff for two different w_max on the same workspace; each result
    # bit-identical to the oracle's quantile of that w_max, and the bins to
    # its bins
    import paper_2511_02510_amd as lv
    import torch
    scene = small_shell(30000, seed=24, lmin=5, lmax=9, clutter=0.1)
    cams = synth.make_cameras_ring(np.random.default_rng(2), 3)
    cams = [look_at(c.o, c.width // 8, c.height // 8) for c in cams]
    say("depth binning then cutoff twice, 30k voxels, 3 views")
    vox = lv.Voxels.from_scene(scene, ctx.device)
    frame = lv.Frame(cams, ctx.device)
    nb = 12
    ws = torch.empty(lv.quantile_workspace_size(vox.n, nb), dtype=torch.uint8, device=ctx.device)
    ws.fill_(0xA5)   # stale contents must not matter
    tau = torch.empty(nb, device=ctx.device)
    prune = torch.empty(vox.n, dtype=torch.uint8, device=ctx.device)
    bins = torch.empty(vox.n, dtype=torch.uint8, device=ctx.device)
    lv.depth_bins(ctx, vox, frame, nb, ws, bins)
    rng = np.random.default_rng(25)
    for q, wm in [(0.1, rng.random(scene.n).astype(np.float32)),
                  (0.3, np.round(rng.random(scene.n) * 8).astype(np.float32) / 8)]:
        lv.depth_cutoff(ctx, vox, to_dev(wm, ctx.device), nb, q, ws, tau, prune)
        torch.cuda.synchronize()
        ref = oquant.depth_quantile(scene, cams, wm, nb, q)
        assert np.array_equal(bins.cpu().numpy(), ref["bins"])
        assert np.array_equal(tau.cpu().numpy(), ref["tau"])
        assert np.array_equal(prune.cpu().numpy(), ref["prune"])
    with pytest.raises(lv.LiteVoxelError):
        lv.depth_bins(ctx, vox, frame, 65, ws)
    with pytest.raises(lv.LiteVoxelError):
        lv.depth_cutoff(ctx, vox, to_dev(wm, ctx.device), nb, 0.0, ws, tau, prune)


def test_depth_quantile_degenerate_inputs(ctx):
    import paper_2511_02510_amd as lv
    import torch
    # every voxel at the same depth proxy (p95 = p5) and tied w_max values
    rng = np.random.default_rng(23)
    scene = synth.make_scene_grid(rng, res_level=2, sh_degree=0)
    cams = [look_at((0.0, 0.0, 3.0), 16, 16)]
    vox = lv.Voxels.from_scene(scene, ctx.device)
    frame = lv.Frame(cams, ctx.device)
    wm = np.zeros(scene.n, np.float32)
    wm[::3] = 0.5
    say("depth quantile degenerate: ties and an empty-bin layout")
    ws = torch.empty(lv.quantile_workspace_size(vox.n, 8), dtype=torch.uint8, device=ctx.device)
    tau = torch.empty(8, device=ctx.device)
    prune = torch.empty(vox.n, dtype=torch.uint8, device=ctx.device)
    bins = torch.empty(vox.n, dtype=torch.uint8, device=ctx.device)
    lv.depth_quantile(ctx, vox, frame, to_dev(wm, ctx.device), 8, 0.25, ws, tau, prune, bins)
    torch.cuda.synchronize()
    ref = oquant.depth_quantile(scene, cams, wm, 8, 0.25)
    assert np.array_equal(bins.cpu().numpy(), ref["bins"])
    assert np.array_equal(tau.cpu().numpy(), ref["tau"])
    assert np.array_equal(prune.cpu().numpy(), ref["prune"])


@pytest.mark.parametrize("n_bins,q", [(1, 0.1), (64, 0.1), (16, 1.0), (5, 0.5)])
def test_depth_quantile_bin_counts_and_ranks(ctx, n_bins, q):
    # one bin (a plain quantile), the largest bin count the entry point takes,
    # the maximum rank (q = 1), and an odd bin count; random w_max with ties
    import paper_2511_02510_amd as lv
    import torch
    scene = small_shell(30000, seed=31, lmin=5, lmax=9, clutter=0.1)
    cams = [look_at((2.2, 0.8, 1.1), 40, 30), look_at((-1.7, 1.3, 1.9), 30, 40)]
    rng = np.random.default_rng(32)
    wm = np.round(rng.random(scene.n) ** 2, 3).astype(np.float32)
    say(f"depth quantile: {n_bins} bins, q = {q}")
    vox = lv.Voxels.from_scene(scene, ctx.device)
    frame = lv.Frame(cams, ctx.device)
    ws = torch.empty(lv.quantile_workspace_size(vox.n, n_bins), dtype=torch.uint8, device=ctx.device)
    tau = torch.empty(n_bins, device=ctx.device)
    prune = torch.empty(vox.n, dtype=torch.uint8, device=ctx.device)
    bins = torch.empty(vox.n, dtype=torch.uint8, device=ctx.device)
    for _ in range(2):   # the second call reuses the workspace as it was left
        lv.depth_quantile(ctx, vox, frame, to_dev(wm, ctx.device), n_bins, q, ws, tau, prune, bins)
    torch.cuda.synchronize()
    ref = oquant.depth_quantile(scene, cams, wm, n_bins, q)
    assert np.array_equal(bins.cpu().numpy(), ref["bins"])
    assert np.array_equal(tau.cpu().numpy(), ref["tau"])
    assert np.array_equal(prune.cpu().numpy(), ref["prune"])


def test_depth_quantile_without_voxels(ctx):
    import paper_2511_02510_amd as lv
    import torch
    say("depth quantile: no voxels")
    scene = synth.scene_subset(small_shell(1000, seed=33, lmin=4, lmax=6), np.arange(0))
    cams = [look_at((2.0, 1.0, 1.5), 16, 16)]
    vox = lv.Voxels.from_scene(scene, ctx.device)
    frame = lv.Frame(cams, ctx.device)
    ws = torch.empty(max(lv.quantile_workspace_size(0, 16), 1), dtype=torch.uint8, device=ctx.device)
    tau = torch.zeros(16, device=ctx.device)
    prune = torch.empty(1, dtype=torch.uint8, device=ctx.device)
    lv.depth_quantile(ctx, vox, frame, torch.empty(1, device=ctx.device), 16, 0.1, ws, tau, prune)
    torch.cuda.synchronize()
    assert np.all(np.isneginf(tau.cpu().numpy()))


def test_autograd_function_matches_direct_calls(ctx):
    import paper_2511_02510_amd as lv
    import torch
    scene = small_shell(8000, seed=24, lmin=5, lmax=8)
    cams = [look_at((2.0, 0.9, 1.0), 48, 40), look_at((-1.0, -1.5, 1.9), 40, 48)]
    say("autograd function")
    vox = lv.Voxels.from_scene(scene, ctx.device)
    frame = lv.Frame(cams, ctx.device)
    r = lv.Renderer(ctx, vox, frame, lv.settings())
    dens = vox.density.clone().requires_grad_(True)
    sh = vox.sh.clone().requires_grad_(True)
    wmax = torch.zeros(vox.n, device=ctx.device)
    rgb, depth, alpha = lv.rasterize(dens, sh, r, wmax)
    rng = np.random.default_rng(25)
    gr, gd, ga = random_grads(rng, frame.P)
    (rgb * to_dev(gr, ctx.device)).sum().backward(retain_graph=True)
    dd_ref, dsh_ref = oracle.backward(scene, cams, gr)
    assert rel_l2(dens.grad.cpu().numpy(), dd_ref) <= GRAD_TOL
    assert rel_l2(sh.grad.cpu().numpy(), dsh_ref) <= GRAD_TOL
    dens.grad = None
    sh.grad = None
    loss = (rgb * to_dev(gr, ctx.device)).sum() + (depth * to_dev(gd, ctx.device)).sum() + \
        (alpha * to_dev(ga, ctx.device)).sum()
    loss.backward()
    dd_ref, dsh_ref = oracle.backward(scene, cams, gr, gd, ga)
    assert rel_l2(dens.grad.cpu().numpy(), dd_ref) <= GRAD_TOL
    assert rel_l2(sh.grad.cpu().numpy(), dsh_ref) <= GRAD_TOL


def test_two_passes_on_one_renderer_backward_together(ctx):
    """Two rasterize calls with different densities (and SH) on one renderer,
    then one backward through both outputs: each node differentiates its own
    pass (saved state per pass), matching the oracle on each scene."""
    import paper_2511_02510_amd as lv
    import torch
    scene = small_shell(6000, seed=26, lmin=5, lmax=8)
    cams = [look_at((1.8, 1.1, 1.2), 44, 36), look_at((-1.2, -1.4, 1.8), 36, 44)]
    say("two autograd passes on one renderer")
    rng = np.random.default_rng(27)
    scene2 = synth.Scene(root_min=scene.root_min, root_size=scene.root_size, ijk=scene.ijk,
                         level=scene.level,
                         density=(scene.density * rng.uniform(0.3, 1.7, scene.density.shape)
                                  ).astype(np.float32),
                         sh=(scene.sh + rng.normal(0, 0.05, scene.sh.shape)).astype(np.float32),
                         sh_degree=scene.sh_degree)
    vox = lv.Voxels.from_scene(scene, ctx.device)
    frame = lv.Frame(cams, ctx.device)
    r = lv.Renderer(ctx, vox, frame, lv.settings(pair_capacity=64))   # the first pass re-plans
    d1 = to_dev(scene.density, ctx.device).requires_grad_(True)
    s1 = to_dev(scene.sh, ctx.device).requires_grad_(True)
    d2 = to_dev(scene2.density, ctx.device).requires_grad_(True)
    s2 = to_dev(scene2.sh, ctx.device).requires_grad_(True)
    wmax = torch.zeros(vox.n, device=ctx.device)
    rgb1, depth1, alpha1 = lv.rasterize(d1, s1, r, wmax)
    rgb2, depth2, alpha2 = lv.rasterize(d2, s2, r, wmax)
    g1 = random_grads(rng, frame.P)
    g2 = random_grads(rng, frame.P)
    loss = sum((o * to_dev(g, ctx.device)).sum()
               for o, g in zip((rgb1, depth1, alpha1, rgb2, depth2, alpha2), g1 + g2))
    loss.backward()
    torch.cuda.synchronize()
    for dens, sh, sc, g, rgb in ((d1, s1, scene, g1, rgb1), (d2, s2, scene2, g2, rgb2)):
        ref = oracle.render(sc, cams)
        assert np.abs(rgb.detach().cpu().numpy() - ref["rgb"]).max() <= IMG_TOL
        dd_ref, dsh_ref = oracle.backward(sc, cams, *g)
        e_d = rel_l2(dens.grad.cpu().numpy(), dd_ref)
        e_s = rel_l2(sh.grad.cpu().numpy(), dsh_ref)
        say(f"  rel-L2 density {e_d:.2e} sh {e_s:.2e}")
        assert e_d <= GRAD_TOL and e_s <= GRAD_TOL
    # the renderer's own buffer was not used by either node
    assert r.st.pair_capacity > 64


def test_graph_replays_match_eager(ctx):
    """fwd + loss + bwd captured once; replays with eager work between them and
    with a moved camera match eager runs."""
    import paper_2511_02510_amd as lv
    import torch
    scene = small_shell(20000, seed=26, lmin=5, lmax=9)
    cams = [look_at((2.1, 0.5, 1.0), 64, 48), look_at((-0.6, 1.2, 2.1), 96, 40)]
    moved = [look_at((2.0, 0.7, 1.2), 64, 48), look_at((-0.7, 1.1, 2.2), 96, 40)]
    rng = np.random.default_rng(27)
    targets = [synth.make_target(rng, c.width, c.height) for c in cams]
    dev = ctx.device
    vox = lv.Voxels.from_scene(scene, dev)
    frame = lv.Frame(cams, dev)
    r = lv.Renderer(ctx, vox, frame, lv.settings(tile=16, chunk=64))
    tgt = to_dev(np.concatenate([t.ravel() for t in targets]), dev)
    rgb, depth, alpha = r.new_outputs()
    wmax = torch.zeros(vox.n, device=dev)
    weight = torch.empty(frame.P, device=dev)
    lws = torch.empty(lv.lf_weight_workspace_size(2), dtype=torch.uint8, device=dev)
    loss = torch.empty(2, device=dev)
    d_rgb = torch.empty(3 * frame.P, device=dev)
    dd = torch.empty_like(vox.density)
    dsh = torch.empty_like(vox.sh)
    stream = torch.cuda.Stream()

    def step():
        wmax.zero_()
        r.forward(rgb, depth, alpha, wmax, stream=stream, verify=False)
        lv.lf_weight(ctx, frame, tgt, 0.5, 1, 1e-3, weight, lws, stream=stream)
        lv.l1_grad(ctx, frame, rgb, tgt, weight, loss, d_rgb, stream=stream)
        r.backward(d_rgb, None, None, dd, dsh, stream=stream)

    def snap():
        torch.cuda.synchronize()
        return [x.clone() for x in (rgb, depth, alpha, wmax, loss, dd, dsh)]

    say("graph capture and replays")
    with torch.cuda.stream(stream):
        r.forward(rgb, depth, alpha, wmax, stream=stream, verify=True)   # size capacity (syncs)
        step()
    eager = snap()
    with torch.cuda.stream(stream):
        lv.graph_begin(ctx, stream)
        step()
        lv.graph_end(ctx, stream)
    for rep in range(3):
        for x in (rgb, depth, dd):
            x.fill_(-7.0)
        torch.cuda.synchronize()
        lv.graph_launch(ctx, stream)
        got = snap()
        for a, b in zip(got[:4], eager[:4]):          # rgb, depth, alpha, w_max: deterministic
            assert torch.equal(a, b), f"replay {rep}"
        # the loss sums block partials with atomics, in scheduling order
        assert torch.allclose(got[4], eager[4], rtol=1e-6, atol=0.0), f"replay {rep}"
        for a, b in zip(got[5:], eager[5:]):
            assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) < 1e-5
        _ = (torch.randn(1000, device=dev) * 2).sum().item()           # eager work between replays
    # move the cameras: the same graph reads the new poses
    frame.set_poses(moved)
    torch.cuda.synchronize()
    lv.graph_launch(ctx, stream)
    got = snap()
    lv.graph_reset(ctx)
    ref = oracle.render(scene, moved)
    assert np.abs(got[0].cpu().numpy() - ref["rgb"]).max() <= IMG_TOL


def test_two_stream_graph_matches_eager(ctx):
    """The step as the benchmark arranges it: the loss weight and the depth
    quantile's binning on a second stream beside the forward, the quantile's
    cutoff beside the L1 gradient, joined by events and captured in one
    graph: every replay (with eager work between them) equals the one-stream
    eager step, which runs the whole quantile in one call."""
    import paper_2511_02510_amd as lv
    import torch
    scene = small_shell(20000, seed=29, lmin=5, lmax=9, clutter=0.1)
    cams = [look_at((2.1, 0.5, 1.0), 80, 60), look_at((-0.6, 1.2, 2.1), 96, 40)]
    rng = np.random.default_rng(30)
    targets = [synth.make_target(rng, c.width, c.height) for c in cams]
    dev = ctx.device
    vox = lv.Voxels.from_scene(scene, dev)
    frame = lv.Frame(cams, dev)
    r = lv.Renderer(ctx, vox, frame, lv.settings(tile=16, chunk=64))
    tgt = to_dev(np.concatenate([t.ravel() for t in targets]), dev)
    rgb, depth, alpha = r.new_outputs()
    wmax = torch.zeros(vox.n, device=dev)
    weight = torch.empty(frame.P, device=dev)
    lws = torch.empty(lv.lf_weight_workspace_size(2), dtype=torch.uint8, device=dev)
    loss = torch.empty(2, device=dev)
    d_rgb = torch.empty(3 * frame.P, device=dev)
    dd = torch.empty_like(vox.density)
    dsh = torch.empty_like(vox.sh)
    qws = torch.empty(lv.quantile_workspace_size(vox.n, 16), dtype=torch.uint8, device=dev)
    tau = torch.empty(16, device=dev)
    prune = torch.empty(vox.n, dtype=torch.uint8, device=dev)
    stream, side = torch.cuda.Stream(), torch.cuda.Stream()

    def step(overlap):
        wmax.zero_()
        aux = side if overlap else stream
        if overlap:
            e0 = torch.cuda.Event()
            e0.record(stream)
            side.wait_event(e0)
        lv.lf_weight(ctx, frame, tgt, 0.5, 1, 1e-3, weight, lws, stream=aux)
        if overlap:
            e_w = torch.cuda.Event()
            e_w.record(side)
            lv.depth_bins(ctx, vox, frame, 16, qws, stream=side)   # needs no w_max
        r.forward(rgb, depth, alpha, wmax, stream=stream, verify=False)
        if overlap:
            e_f = torch.cuda.Event()
            e_f.record(stream)
            stream.wait_event(e_w)
            side.wait_event(e_f)
            lv.depth_cutoff(ctx, vox, wmax, 16, 0.1, qws, tau, prune, stream=side)
            e_q = torch.cuda.Event()
            e_q.record(side)
        else:
            lv.depth_quantile(ctx, vox, frame, wmax, 16, 0.1, qws, tau, prune, stream=stream)
        lv.l1_grad(ctx, frame, rgb, tgt, weight, loss, d_rgb, stream=stream)
        if overlap:
            stream.wait_event(e_q)
        r.backward(d_rgb, None, None, dd, dsh, stream=stream)

    def snap():
        torch.cuda.synchronize()
        return [x.clone() for x in (rgb, depth, alpha, wmax, loss, weight, tau, prune, dd, dsh)]

    say("two-stream graph capture and replays")
    with torch.cuda.stream(stream):
        r.forward(rgb, depth, alpha, wmax, stream=stream, verify=True)   # size capacity (syncs)
        step(False)
    eager = snap()
    with torch.cuda.stream(stream):
        lv.graph_begin(ctx, stream)
        step(True)
        lv.graph_end(ctx, stream)
    for rep in range(3):
        for x in (rgb, weight, tau, dd):
            x.fill_(-7.0)
        prune.fill_(9)
        torch.cuda.synchronize()
        lv.graph_launch(ctx, stream)
        got = snap()
        for i in (0, 1, 2, 3, 6, 7):                  # rgb, depth, alpha, w_max, tau, prune
            assert torch.equal(got[i], eager[i]), f"replay {rep}, output {i}"
        # the loss and the weight normalisation sum block partials with atomics
        for i in (4, 5):
            assert torch.allclose(got[i], eager[i], rtol=1e-6, atol=0.0), f"replay {rep}, output {i}"
        for a, b in zip(got[8:], eager[8:]):
            assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) < 1e-5
        _ = (torch.randn(1000, device=dev) * 2).sum().item()           # eager work between replays
    lv.graph_reset(ctx)


def test_autotune_returns_a_runnable_setting(ctx, tmp_path):
    import paper_2511_02510_amd as lv
    scene = small_shell(20000, seed=28, lmin=5, lmax=9)
    cams = [look_at((2.1, 0.5, 1.0), 160, 120)]
    say("autotune")
    vox = lv.Voxels.from_scene(scene, ctx.device)
    frame = lv.Frame(cams, ctx.device)
    cache = str(tmp_path / "tune.json")
    best, table = lv.autotune(ctx, vox, frame, reps=2, cache=cache)
    again, table2 = lv.autotune(ctx, vox, frame, reps=2, cache=cache)   # served by the cache
    assert (again.tile, again.chunk, again.chunk_bwd) == (best.tile, best.chunk, best.chunk_bwd)
    assert np.allclose(table2, np.round(table, 4))
    assert best.tile in (8, 16, 32) and best.chunk in (64, 128, 256) and best.chunk_bwd in (64, 128, 256)
    assert table.shape == (2, 3, 3) and np.all(table > 0)
    # the chosen tile minimises fastest forward + fastest backward; the chunks are those minima
    ti = [8, 16, 32].index(best.tile)
    per_tile = table[0].min(axis=1) + table[1].min(axis=1)
    assert abs(per_tile.min() - per_tile[ti]) < 1e-9
    assert table[0, ti, [64, 128, 256].index(best.chunk)] == table[0, ti].min()
    assert table[1, ti, [64, 128, 256].index(best.chunk_bwd)] == table[1, ti].min()
    g = run_gpu(ctx, scene, cams, tile=best.tile, chunk=best.chunk, cap=best.pair_capacity, export=False)
    ref = oracle.render(scene, cams)
    assert np.abs(g["rgb"] - ref["rgb"]).max() <= IMG_TOL
