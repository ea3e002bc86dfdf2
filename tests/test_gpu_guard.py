"""GPU parity of the pruning stability guards (Sec. IV-C, guards i-iii)
through the C-ABI: prune mask, moving average and in/out state bit-exact
against the oracle over consecutive adaptation steps, with the quantile
inputs (bins, tau) themselves checked bit-exact first."""
import math

import numpy as np
import pytest

import synth
from oracle import guard as oguard
from oracle import quantile as oquant
from synth.scenes import Scene, look_at
from gpu_helpers import say, small_shell, to_dev

pytestmark = pytest.mark.gpu

f32 = np.float32


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_02510_amd as lv
    c = lv.Context(0)
    yield c
    c.close()


class GuardRun:
    """Device buffers of one scene: quantile, then guard steps."""

    def __init__(self, ctx, scene, cams, n_bins):
        import paper_2511_02510_amd as lv
        import torch
        self.lv, self.torch, self.ctx = lv, torch, ctx
        dev = ctx.device
        self.scene, self.cams, self.n_bins = scene, cams, n_bins
        self.vox = lv.Voxels.from_scene(scene, dev)
        self.frame = lv.Frame(cams, dev)
        n = scene.n
        self.qws = torch.empty(max(lv.quantile_workspace_size(n, n_bins), 1), dtype=torch.uint8, device=dev)
        self.gws = torch.empty(max(lv.guard_workspace_size(n), 1), dtype=torch.uint8, device=dev)
        self.tau = torch.empty(n_bins, device=dev)
        self.qprune = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
        self.bins = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
        self.ema = torch.ones(max(n, 1), device=dev)
        self.state = torch.ones(max(n, 1), dtype=torch.uint8, device=dev)
        self.prune = torch.full((max(n, 1),), 7, dtype=torch.uint8, device=dev)
        self.npr = torch.full((1,), 12345, dtype=torch.int32, device=dev)

    def quantile(self, wmax, q):
        self.wmax = to_dev(wmax, self.ctx.device)
        self.lv.depth_quantile(self.ctx, self.vox, self.frame, self.wmax, self.n_bins, q, self.qws,
                               self.tau, self.qprune, self.bins)

    def step(self, **params):
        self.lv.prune_guard(self.ctx, self.vox, self.frame, self.wmax, self.bins, self.tau,
                            self.n_bins, self.lv.guard_params(**params), self.gws, self.ema,
                            self.state, self.prune, self.npr)
        self.torch.cuda.synchronize()
        n = self.scene.n
        return (self.prune.cpu().numpy()[:n], self.ema.cpu().numpy()[:n],
                self.state.cpu().numpy()[:n], int(self.npr.cpu().numpy()[0]))


def _steps(ctx, scene, cams, n_bins, wmaxes, q, params, ema0=None, state0=None):
    run = GuardRun(ctx, scene, cams, n_bins)
    n = scene.n
    m = np.ones(n, f32) if ema0 is None else ema0.astype(f32)
    s = np.ones(n, np.uint8) if state0 is None else state0.astype(np.uint8)
    if n:
        run.ema.copy_(to_dev(m, ctx.device))
        run.state.copy_(to_dev(s, ctx.device, np.uint8))
    delta = oquant.depth_proxy(scene, cams)
    bins_ref, _, _ = oquant.depth_bins(delta, n_bins)
    pruned = 0
    for t, wm in enumerate(wmaxes):
        run.quantile(wm, q)
        tau_ref, _ = oquant.quantile_cutoffs(wm, bins_ref, n_bins, q)
        assert np.array_equal(run.bins.cpu().numpy()[:n], bins_ref), "bins"
        assert np.array_equal(run.tau.cpu().numpy(), tau_ref), "tau"
        pr, em, st, npr = run.step(**params)
        ref_pr, m, s = oguard.guard_step(scene, cams, wm, bins_ref, tau_ref, m, s, **params)
        assert np.array_equal(em.view(np.uint32), m.view(np.uint32)), f"ema, step {t}"
        assert np.array_equal(st, s), f"state, step {t}"
        assert np.array_equal(pr, ref_pr), f"prune, step {t}"
        assert npr == int(ref_pr.sum())
        pruned += npr
    return pruned


def test_guard_steps_shell(ctx):
    scene = small_shell(30000, seed=31, lmin=5, lmax=10, clutter=0.15)
    cams = [look_at((2.0, 0.8, 1.1), 96, 72), look_at((-1.2, 0.4, -2.0), 80, 64)]
    rng = np.random.default_rng(32)
    wms = [(rng.uniform(0, 1, scene.n) ** 3).astype(f32) for _ in range(4)]
    for wm in wms:
        wm[rng.random(scene.n) < 0.2] = 0.0
    say("guards: 30k voxels, 4 steps, default constants")
    assert _steps(ctx, scene, cams, 16, wms, 0.3, {}) > 0
    say("guards: a binding cap, strong halo")
    p = dict(alpha=0.5, m_low=0.4, m_high=0.6, rho=0.6, w_keep=0.3, cap_frac=0.004)
    assert _steps(ctx, scene, cams, 8, wms, 0.5, p) > 0


def test_guard_cap_ties_taken_in_index_order(ctx):
    # every voxel starts with the same average and fails the quantile test, so
    # all averages stay equal and the cap picks the lowest indices
    rng = np.random.default_rng(33)
    scene = synth.make_scene_grid(rng, res_level=5, sh_degree=0)   # 32^3 voxels
    cams = [look_at((2.3, 1.5, 2.7), 64, 64)]
    wm = np.zeros(scene.n, f32)
    p = dict(alpha=0.5, m_low=0.6, m_high=0.9, rho=0.0, w_keep=2.0, cap_frac=0.1)
    say("guards: ties at the cap, 32768 voxels")
    run = GuardRun(ctx, scene, cams, 4)
    run.quantile(wm, 0.5)
    pr, em, st, npr = run.step(**p)
    cap = math.floor(0.1 * scene.n)
    assert npr == cap and np.all(em == 0.5) and np.all(st == 0)
    assert np.array_equal(np.nonzero(pr)[0], np.arange(cap))
    # the next step: the same tie, the same cap, the same lowest indices
    pr2, em2, _, npr2 = run.step(**p)
    assert npr2 == cap and np.all(em2 == 0.25) and np.array_equal(np.nonzero(pr2)[0], np.arange(cap))


@pytest.mark.parametrize("cap_frac", [0.0, 1.0])
def test_guard_cap_extremes(ctx, cap_frac):
    scene = small_shell(8000, seed=34, lmin=4, lmax=8, clutter=0.2)
    cams = [look_at((1.9, -0.6, 1.4), 64, 48)]
    rng = np.random.default_rng(35)
    wms = [(rng.uniform(0, 1, scene.n) ** 2).astype(f32) for _ in range(3)]
    say(f"guards: cap_frac {cap_frac}")
    p = dict(alpha=0.6, m_low=0.5, m_high=0.8, rho=0.1, w_keep=0.9, cap_frac=cap_frac)
    got = _steps(ctx, scene, cams, 4, wms, 0.4, p)
    assert (got == 0) == (cap_frac == 0.0)


def test_guard_without_voxels_and_argument_errors(ctx):
    import paper_2511_02510_amd as lv
    empty = Scene(root_min=np.array([-1, -1, -1], np.float32), root_size=2.0,
                  ijk=np.zeros((3, 0), np.uint16), level=np.zeros(0, np.uint8),
                  density=np.zeros((8, 0), np.float32), sh=np.zeros((3, 0), np.float32), sh_degree=0)
    cams = [look_at((2.0, 1.0, 1.5), 8, 8)]
    say("guards: no voxels, bad arguments")
    run = GuardRun(ctx, empty, cams, 4)
    run.quantile(np.zeros(0, f32), 0.1)
    _, _, _, npr = run.step()
    assert npr == 0
    scene = small_shell(2000, seed=36, lmin=4, lmax=7)
    run = GuardRun(ctx, scene, cams, 4)
    run.quantile(np.zeros(scene.n, f32), 0.1)
    for bad in (dict(alpha=0.0), dict(alpha=1.5), dict(m_low=0.8, m_high=0.2), dict(rho=-1.0),
                dict(cap_frac=1.5), dict(cap_frac=-0.1)):
        with pytest.raises(lv.LiteVoxelError):
            run.step(**bad)
    assert np.all(run.prune.cpu().numpy() == 7)   # nothing was enqueued


def test_guard_fullsize_ring(ctx):
    # the benchmark's 1M-voxel scene and 8 views, w_max from its forward pass
    import paper_2511_02510_amd as lv
    import torch
    scene, cams, _ = synth.make_config("ring1m")
    say("guards: 1M voxels, 8 views, 3 steps")
    vox = lv.Voxels.from_scene(scene, ctx.device)
    frame = lv.Frame(cams, ctx.device)
    r = lv.Renderer(ctx, vox, frame, lv.settings())
    rgb, depth, alpha = r.new_outputs()
    wmax = torch.zeros(vox.n, device=ctx.device)
    r.forward(rgb, depth, alpha, wmax)
    torch.cuda.synchronize()
    w0 = wmax.cpu().numpy().astype(f32)
    rng = np.random.default_rng(37)
    wms = [w0, (w0 * rng.uniform(0.5, 1.0, scene.n)).astype(f32), (w0 ** 1.5).astype(f32)]
    # default constants: a voxel needs four failed quantile tests in a row to
    # turn out, so nothing is pruned in three steps
    assert _steps(ctx, scene, cams, 16, wms, 0.1, {}) == 0
    # alpha 1/2: out after two, then capped at 2% of the voxels
    assert _steps(ctx, scene, cams, 16, wms, 0.1, dict(alpha=0.5, cap_frac=0.02)) > 0
