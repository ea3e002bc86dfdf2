"""GPU parity of one adaptation cycle of the training loop (Sec. IV-A loop,
Sec. IV-C pruning with its guards, Sec. IV-D subdivision) as the trainer runs
it: per-bin quantile -> guards -> compaction of the kept voxels and of their
per-voxel state -> footprint percentiles -> budgeted selection -> 8-way
split.  The refined voxel set (ijk, level, densities, SH), the moving
averages (bit patterns) and the in/out state are compared bit-exactly with
the oracle chain on the same seeded inputs, then the refined set is rendered
by both sides at the image bars."""
import numpy as np
import pytest

import oracle
from oracle import guard as oguard
from oracle import quantile as oquant
from oracle import split as osplit
from synth.scenes import Scene, look_at
from gpu_helpers import IMG_TOL, WMAX_TOL, check_images, say, small_shell, to_dev

pytestmark = pytest.mark.gpu

f32 = np.float32


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_02510_amd as lv
    c = lv.Context(0)
    yield c
    c.close()


def oracle_cycle(scene, cams, wmax, useful, ema, state, n_bins, q, guard, split):
    """The adaptation cycle written out with the oracle's functions and numpy
    compaction; returns the refined scene, its averages and states, and the
    intermediate decisions."""
    dq = oquant.depth_quantile(scene, cams, wmax, n_bins, q)
    prune, m, s = oguard.guard_step(scene, cams, wmax, dq["bins"], dq["tau"], ema, state, **guard)
    keep = prune == 0
    kept = Scene(root_min=scene.root_min.copy(), root_size=scene.root_size,
                 ijk=scene.ijk[:, keep].copy(), level=scene.level[keep].copy(),
                 density=scene.density[:, keep].copy(), sh=scene.sh[:, keep].copy(),
                 sh_degree=scene.sh_degree)
    z5, z95 = osplit.footprint_range(kept, cams)
    flags, _, _ = osplit.select(kept, cams, useful[keep], z5, z95, **split)
    refined = osplit.apply_split(kept, flags)
    eff = flags.astype(bool) & (kept.level.astype(np.int32) < osplit.L_MAX)
    reps = np.where(eff, 8, 1)
    return dict(scene=refined, ema=np.repeat(m[keep], reps), state=np.repeat(s[keep], reps),
                pruned=int((~keep).sum()), split=int(eff.sum()), tau=dq["tau"])


def run_trainer_cycle(ctx, scene, cams, wmax, useful, ema, state, n_bins, q, guard, split):
    import torch
    import paper_2511_02510_amd as lv
    from paper_2511_02510_amd.train import TrainConfig, Trainer
    dev = ctx.device
    vox = lv.Voxels.from_scene(scene, dev)
    frame = lv.Frame(cams, dev)
    target = torch.zeros(3 * frame.P, device=dev)
    cfg = TrainConfig(prune="depth_quantile", n_bins=n_bins, q=q, guard=dict(guard),
                      split=dict(split))
    tr = Trainer(ctx, vox, frame, target, cfg)
    tr.wmax = to_dev(wmax, dev)
    tr.useful = to_dev(useful, dev)
    tr.ema = to_dev(ema, dev)
    tr.state = to_dev(state, dev, np.uint8)
    rec = tr.adapt()
    torch.cuda.synchronize()
    return tr, rec


def _inputs(rng, scene, cams):
    # w_max of the unsplit scene as the oracle renders it, a fifth of it set
    # to exact zeros (ties at the cutoffs); usefulness with zeros; averages
    # and states drawn at random (some at the hysteresis thresholds)
    wmax = oracle.render(scene, cams)["wmax"].astype(f32)
    wmax[rng.random(scene.n) < 0.2] = 0.0
    useful = (rng.uniform(0, 1, scene.n) ** 2).astype(f32)
    useful[rng.random(scene.n) < 0.3] = 0.0
    ema = rng.uniform(0, 1, scene.n).astype(f32)
    ema[rng.random(scene.n) < 0.1] = f32(0.3)
    state = (rng.random(scene.n) < 0.6).astype(np.uint8)
    return wmax, useful, ema, state


CASES = {
    "default_guards": (dict(), dict(max_splits=400)),
    "binding_cap_kappa_half": (dict(alpha=0.5, m_low=0.4, m_high=0.6, rho=0.1, w_keep=0.9,
                                    cap_frac=0.01), dict(kappa=0.5, beta=0.5, max_splits=150)),
    "neutral_guards": (dict(alpha=1.0, m_low=0.5, m_high=0.5, rho=0.0, w_keep=2.0, cap_frac=1.0),
                       dict(max_splits=8192)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_adaptation_cycle_matches_oracle_chain(ctx, case):
    import torch
    guard, split = CASES[case]
    scene = small_shell(20000, seed=71, deg=1, lmin=4, lmax=9, clutter=0.1)
    cams = [look_at((2.1, 0.9, 1.2), 128, 96), look_at((-1.4, 0.5, -1.9), 112, 80)]
    rng = np.random.default_rng(72)
    wmax, useful, ema, state = _inputs(rng, scene, cams)
    n_bins, q = 16, 0.2
    say(f"adaptation cycle [{case}]: {scene.n} voxels, 2 views")
    ref = oracle_cycle(scene, cams, wmax, useful, ema, state, n_bins, q, guard, split)
    tr, rec = run_trainer_cycle(ctx, scene, cams, wmax, useful, ema, state, n_bins, q, guard, split)
    say(f"  oracle pruned {ref['pruned']} split {ref['split']}; trainer {rec}")
    assert rec["pruned"] == ref["pruned"] and rec["split"] == ref["split"]
    assert ref["pruned"] > 0 and ref["split"] > 0
    out = ref["scene"]
    assert rec["voxels"] == out.n == tr.vox.n
    assert np.array_equal(tr.vox.ijk.cpu().numpy().astype(np.uint16), out.ijk), "ijk"
    assert np.array_equal(tr.vox.level.cpu().numpy(), out.level), "level"
    assert np.array_equal(tr.density.detach().cpu().numpy().view(np.uint32),
                          out.density.astype(f32).view(np.uint32)), "densities"
    assert np.array_equal(tr.sh.detach().cpu().numpy().view(np.uint32),
                          out.sh.astype(f32).view(np.uint32)), "SH"
    assert np.array_equal(tr.ema.cpu().numpy().view(np.uint32), ref["ema"].view(np.uint32)), "ema"
    assert np.array_equal(tr.state.cpu().numpy(), ref["state"]), "state"
    # the refined set renders like the oracle's (fresh w_max window)
    tr.renderer.forward(tr.rgb, tr.depth, tr.alpha, tr.wmax)
    torch.cuda.synchronize()
    got = {"rgb": tr.rgb.cpu().numpy().astype(np.float64),
           "depth": tr.depth.cpu().numpy().astype(np.float64),
           "alpha": tr.alpha.cpu().numpy().astype(np.float64)}
    img = oracle.render(out, cams)
    check_images(got, img)
    e_w = float(np.abs(tr.wmax.cpu().numpy().astype(np.float64)[:out.n] - img["wmax"]).max())
    say(f"  refined set: w_max max abs {e_w:.2e}")
    assert e_w <= WMAX_TOL
