"""The allocation-free loss-weight entry point (lv_lf_weight_noalloc, static
scratch) against lv_lf_weight with a caller workspace, through the C-ABI, on
two calls in a row, the second with a smaller input."""
import numpy as np
import pytest

import synth
from synth.scenes import look_at
from gpu_helpers import say, to_dev

pytestmark = pytest.mark.gpu


def _weights(ctx, cams, targets, gamma, form, eps, noalloc):
    import paper_2511_02510_amd as lv
    import torch
    frame = lv.Frame(cams, ctx.device)
    target = to_dev(np.concatenate([t.ravel() for t in targets]), ctx.device)
    weight = torch.full((frame.P,), float("nan"), device=ctx.device)
    if noalloc:
        lv.lf_weight_noalloc(ctx, frame, target, gamma, form, eps, weight)
    else:
        ws = torch.empty(lv.lf_weight_workspace_size(frame.n_views), dtype=torch.uint8,
                         device=ctx.device)
        lv.lf_weight(ctx, frame, target, gamma, form, eps, weight, ws)
    torch.cuda.synchronize()
    return weight.cpu().numpy()


def test_noalloc_weight_matches_workspace_call():
    import paper_2511_02510_amd as lv
    ctx = lv.Context(0)
    rng = np.random.default_rng(71)
    big = [look_at((2.0, 0.6, 1.3), 320, 240), look_at((-1.5, 1.0, 2.0), 257, 129),
           look_at((0.2, 2.3, -1.1), 96, 200), look_at((1.1, -1.9, 1.2), 64, 48)]
    small = [look_at((0.7, 1.5, -1.8), 45, 33)]
    cases = [(big, 0.6, 0, 1e-3), (small, 1.0, 1, 1e-3)]   # second call: smaller input
    for cams, gamma, form, eps in cases:
        targets = [synth.make_target(rng, c.width, c.height) for c in cams]
        say(f"noalloc lf_weight: {len(cams)} views, form {form}, gamma {gamma}")
        ref = _weights(ctx, cams, targets, gamma, form, eps, noalloc=False)
        got = _weights(ctx, cams, targets, gamma, form, eps, noalloc=True)
        assert np.all(np.isfinite(got))
        # same kernels; the per-view mean is summed with float atomics in
        # arbitrary order, so the normalised weights may differ in the last bits
        err = float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30)))
        say(f"  max rel diff {err:.2e}")
        assert err <= 1e-6
        # the mean normalisation of eq. 8 holds per view
        off = np.cumsum([0] + [c.width * c.height for c in cams])
        for v in range(len(cams)):
            assert abs(got[off[v]:off[v + 1]].mean() - 1.0) < 1e-5
    # more views than the static scratch holds: an argument error, nothing run
    cams = [look_at((2.0, 0.6, 1.3), 8, 8)] * 65
    frame = lv.Frame(cams, ctx.device)
    import torch
    t = torch.zeros(3 * frame.P, device=ctx.device)
    w = torch.zeros(frame.P, device=ctx.device)
    with pytest.raises(lv.LiteVoxelError, match="static scratch"):
        lv.lf_weight_noalloc(ctx, frame, t, 0.5, 0, 1e-3, w)
    ctx.close()
