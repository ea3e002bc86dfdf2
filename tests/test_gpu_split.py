"""GPU parity of priority-driven subdivision (Sec. IV-D, eq. 13-16) and the
8-way split through the C-ABI: footprint percentiles, split selection,
priorities and the refined voxel arrays bit-exact against the oracle; the
refined set rasterizes with keys identical to the oracle's and the same
colour and opacity as the unsplit set."""
import numpy as np
import pytest

import synth
from oracle import split as osplit
from synth.scenes import Scene, look_at
from gpu_helpers import IMG_TOL, check_keys, run_gpu, say, small_shell, to_dev

pytestmark = pytest.mark.gpu

f32 = np.float32


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_02510_amd as lv
    c = lv.Context(0)
    yield c
    c.close()


class SplitRun:
    def __init__(self, ctx, scene, cams):
        import paper_2511_02510_amd as lv
        import torch
        self.lv, self.torch, self.ctx = lv, torch, ctx
        dev = ctx.device
        self.scene, self.cams = scene, cams
        self.vox = lv.Voxels.from_scene(scene, dev)
        self.frame = lv.Frame(cams, dev)
        n = scene.n
        self.ws = torch.empty(max(lv.split_workspace_size(n), 1), dtype=torch.uint8, device=dev)
        self.range = torch.full((2,), -7.0, device=dev)
        self.split = torch.full((max(n, 1),), 9, dtype=torch.uint8, device=dev)
        self.prio = torch.empty(max(n, 1), device=dev)
        self.nsp = torch.full((1,), 12345, dtype=torch.int32, device=dev)
        self.need = torch.full((1,), -1, dtype=torch.int64, device=dev)

    def footprint_range(self):
        self.lv.footprint_range(self.ctx, self.vox, self.frame, self.ws, self.range)
        self.torch.cuda.synchronize()
        return self.range.cpu().numpy()

    def select(self, score, **params):
        self.score = to_dev(score, self.ctx.device)
        self.lv.subdivide_select(self.ctx, self.vox, self.frame, self.score, self.range,
                                 self.lv.split_params(**params), self.ws, self.split, self.prio,
                                 self.nsp)
        self.torch.cuda.synchronize()
        n = self.scene.n
        return (self.split.cpu().numpy()[:n], self.prio.cpu().numpy()[:n],
                int(self.nsp.cpu().numpy()[0]))

    def apply(self, flags, n_out):
        if self.scene.n:
            self.split.copy_(to_dev(flags, self.ctx.device, np.uint8))
        v = self.lv.subdivide_apply(self.ctx, self.vox, self.split, n_out, self.ws, self.need)
        self.torch.cuda.synchronize()
        return v, int(self.need.cpu().numpy()[0])


def _arrays(v):
    return (v.ijk.cpu().numpy().view(np.uint16), v.level.cpu().numpy(), v.density.cpu().numpy(),
            v.sh.cpu().numpy())


def _same_refined(v, ref, rows=None):
    got = _arrays(v)
    want = (ref.ijk, ref.level, ref.density, ref.sh)
    for g, w, name in zip(got, want, ("ijk", "level", "density", "sh")):
        if rows is not None:
            g, w = g[..., :rows], w[..., :rows]
        assert np.array_equal(np.ascontiguousarray(g).view(np.uint8),
                              np.ascontiguousarray(w).view(np.uint8)), name


def test_footprint_range_and_selection(ctx):
    scene = small_shell(30000, seed=41, lmin=5, lmax=11, clutter=0.2)
    cams = [look_at((2.0, 0.8, 1.1), 96, 72), look_at((-1.2, 0.4, -2.0), 80, 64)]
    run = SplitRun(ctx, scene, cams)
    say("subdivision: footprint percentiles, 30k voxels")
    rng_ = run.footprint_range()
    z5, z95 = osplit.footprint_range(scene, cams)
    assert rng_[0] == z5 and rng_[1] == z95
    rng = np.random.default_rng(42)
    for trial, (kappa, beta, k) in enumerate([(1.0, 0.2, 500), (0.3, 0.3, 4000), (0.05, 0.0, 100000),
                                              (2.0, 0.1, 0), (0.5, 0.25, 1)]):
        # ties, zero, negative and NaN scores, and half of them continuous
        score = rng.choice(np.array([0.0, 0.5, 1.0, 1.5, -1.0, np.nan], f32), scene.n)
        cont = rng.random(scene.n) < 0.5
        score[cont] = rng.uniform(0, 2, int(cont.sum())).astype(f32)
        say(f"  select kappa={kappa} beta={beta} max_splits={k}")
        got, prio, ns = run.select(score, kappa=kappa, beta=beta, max_splits=k)
        want, wprio, elig = osplit.select(scene, cams, score, z5, z95, kappa=kappa, beta=beta,
                                          max_splits=k)
        assert np.array_equal(prio.view(np.uint32), wprio.view(np.uint32)), trial
        assert np.array_equal(got, want), trial
        assert ns == int(want.sum())
    assert ns == 1


def test_apply_matches_oracle_and_rasterizes(ctx):
    scene = small_shell(20000, seed=43, lmin=5, lmax=12, clutter=0.2)
    scene.sh = scene.sh[:3].copy()          # SH degree 0: colour independent of the centre
    scene.sh_degree = 0
    cams = [look_at((1.9, 0.7, 1.2), 96, 72), look_at((-0.6, 1.1, -2.1), 80, 60)]
    rng = np.random.default_rng(44)
    flags = (rng.random(scene.n) < 0.25).astype(np.uint8)
    flags[scene.level == 12] = 1            # ignored: the finest level has no children
    ref = osplit.apply_split(scene, flags)
    say(f"subdivision: apply, 20k voxels -> {ref.n}")
    run = SplitRun(ctx, scene, cams)
    v, need = run.apply(flags, ref.n)
    assert need == ref.n and v.n == ref.n
    _same_refined(v, ref)
    # the refined set is a valid input of the rasterizer: keys as the oracle's,
    # and (SH 0) the same colour and opacity as the unsplit set
    say("  refined set through the rasterizer")
    g0 = run_gpu(ctx, scene, cams, export=False)
    g1 = run_gpu(ctx, ref, cams)
    check_keys(g1["bins"], ref, cams, 16)
    assert np.abs(g0["rgb"] - g1["rgb"]).max() <= IMG_TOL
    assert np.abs(g0["alpha"] - g1["alpha"]).max() <= IMG_TOL


def test_apply_truncated_output_and_no_voxels(ctx):
    scene = small_shell(5000, seed=45, lmin=4, lmax=8, clutter=0.1)
    cams = [look_at((2.0, 0.5, 1.3), 32, 24)]
    rng = np.random.default_rng(46)
    flags = (rng.random(scene.n) < 0.3).astype(np.uint8)
    ref = osplit.apply_split(scene, flags)
    run = SplitRun(ctx, scene, cams)
    short = ref.n - 13   # ends inside a split voxel's children (or after)
    say(f"subdivision: output cut at {short} of {ref.n} rows")
    v, need = run.apply(flags, short)
    assert need == ref.n
    _same_refined(v, ref, rows=short)
    empty = Scene(root_min=np.array([-1, -1, -1], np.float32), root_size=2.0,
                  ijk=np.zeros((3, 0), np.uint16), level=np.zeros(0, np.uint8),
                  density=np.zeros((8, 0), np.float32), sh=np.zeros((3, 0), np.float32), sh_degree=0)
    run = SplitRun(ctx, empty, cams)
    assert np.array_equal(run.footprint_range(), [0.0, 0.0])
    _, _, ns = run.select(np.zeros(0, f32))
    assert ns == 0
    v, need = run.apply(np.zeros(0, np.uint8), 0)
    assert need == 0 and v.n == 0


def test_split_argument_errors(ctx):
    import paper_2511_02510_amd as lv
    scene = small_shell(2000, seed=47, lmin=4, lmax=7)
    cams = [look_at((2.0, 0.5, 1.3), 16, 16)]
    run = SplitRun(ctx, scene, cams)
    run.footprint_range()
    say("subdivision: argument errors")
    for bad in (dict(kappa=-1.0), dict(beta=float("nan")), dict(kappa=float("inf"))):
        with pytest.raises(lv.LiteVoxelError):
            run.select(np.ones(scene.n, f32), **bad)
    assert np.all(run.split.cpu().numpy() == 9)   # nothing was enqueued
    for n_out in (scene.n - 1, 8 * scene.n + 1):
        with pytest.raises(lv.LiteVoxelError):
            run.apply(np.zeros(scene.n, np.uint8), n_out)


def test_split_fullsize_ring(ctx):
    # the benchmark's 1M-voxel scene: usefulness = its w_max, 8192 splits
    import paper_2511_02510_amd as lv
    import torch
    scene, cams, _ = synth.make_config("ring1m")
    say("subdivision: 1M voxels, 8 views")
    run = SplitRun(ctx, scene, cams)
    r = lv.Renderer(ctx, run.vox, run.frame, lv.settings())
    rgb, depth, alpha = r.new_outputs()
    wmax = torch.zeros(run.vox.n, device=ctx.device)
    r.forward(rgb, depth, alpha, wmax)
    torch.cuda.synchronize()
    score = wmax.cpu().numpy().astype(f32)
    rng_ = run.footprint_range()
    z5, z95 = osplit.footprint_range(scene, cams)
    assert rng_[0] == z5 and rng_[1] == z95
    got, prio, ns = run.select(score, kappa=1.0, beta=0.2, max_splits=8192)
    want, wprio, _ = osplit.select(scene, cams, score, z5, z95, kappa=1.0, beta=0.2, max_splits=8192)
    assert np.array_equal(prio.view(np.uint32), wprio.view(np.uint32))
    assert np.array_equal(got, want) and ns == int(want.sum()) and ns > 0
    ref = osplit.apply_split(scene, want)
    v, need = run.apply(want, ref.n)
    assert need == ref.n
    _same_refined(v, ref)
