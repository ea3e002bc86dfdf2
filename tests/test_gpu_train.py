"""End-to-end synthetic training through the library (Sec. IV-A loop with the
LF-weighted L1 of eq. 7-10, the eq. 9 ramp, depth-aware pruning with guards,
and priority-driven subdivision): the loss falls, the images approach the
targets, the voxel set is pruned and refined, and the parameters stay finite,
with the depth-quantile pruning and with the global-threshold baseline."""
import numpy as np
import pytest

from gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_02510_amd as lv
    c = lv.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("mode", ["depth_quantile", "global"])
def test_training_loop_converges_and_adapts(ctx, mode):
    import torch
    from paper_2511_02510_amd import train
    vox, frame, target, _, _ = train.training_problem(ctx, n_gt=20000, views=4, res=(128, 96),
                                                      init_level=4, seed=3)
    n0 = vox.n
    cfg = train.TrainConfig(iters=120, adapt_every=40, prune=mode,
                            guard=dict(alpha=0.5, cap_frac=0.2), split=dict(max_splits=2000))
    say(f"training: {mode}, {n0} voxels to start, 120 iterations")
    t = train.Trainer(ctx, vox, frame, target, cfg)
    res = t.run(log=lambda r: say(f"  {r}"))
    say(f"  final loss {res['final_loss']:.4g} (first {res['first_loss']:.4g}), "
        f"PSNR {res['final_psnr']:.2f}, voxels {res['voxels']}, peak {res['peak_vram_mb']} MB")
    assert res["final_loss"] < 0.6 * res["first_loss"]
    assert res["final_psnr"] > res["adapt"][0]["psnr"]
    assert len(res["adapt"]) == 2
    assert sum(a["split"] for a in res["adapt"]) > 0
    assert sum(a["pruned"] for a in res["adapt"]) > 0
    assert res["voxels"] != n0
    assert torch.isfinite(t.density).all() and torch.isfinite(t.sh).all()
    assert t.ema.shape[0] == t.vox.n and t.state.shape[0] == t.vox.n
    lv_ = np.unique(t.vox.level.cpu().numpy())
    assert lv_.min() >= 4 and lv_.max() <= 6          # two rounds of splits from level 4
