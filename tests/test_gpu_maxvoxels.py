"""The largest voxel count the C-ABI takes (n = 2^28 - 1): a slab of
268,432,455 finest-level cells behind the camera (every corner behind the
near plane, so every one is culled) and a 3000-leaf shell in front of it
holding the largest ids, 2^28 - 3001 .. 2^28 - 2.  Voxel ids fill the 28 id
bits of the sort keys and the gradient rows are addressed at the top of
their range, so this pins the id packing and the flush's offsets at the
limit.  The shell alone goes through the FP64 oracle: keys (ids shifted by
the slab's size), images, w_max and gradients must match it, and every slab
voxel must be culled with zero w_max and zero gradients."""
import numpy as np
import pytest

import oracle
from synth.scenes import look_at
from gpu_helpers import (GRAD_TOL, WMAX_TOL, check_images, random_grads, rel_l2, say, small_shell,
                         to_dev)

pytestmark = pytest.mark.gpu

N_MAX = (1 << 28) - 1
SLAB_LEVEL = 12


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_02510_amd as lv
    c = lv.Context(0)
    yield c
    c.close()


def _slab_and_shell(dev):
    """Device arrays of the slab (first) and the shell (last), and the shell
    as a host scene for the oracle."""
    import torch
    shell = small_shell(3000, seed=161, deg=0, lmin=4, lmax=6, clutter=0.0)
    k = shell.n
    m = N_MAX - k
    side = 1 << SLAB_LEVEL
    # level-12 cells x, y in [0, 4096), z in [0, 16): z below -0.992 in the
    # root [-1, 1]^3, under the shell's lowest cell (z >= -0.875)
    assert m <= side * side * 16
    idx = torch.arange(m, device=dev, dtype=torch.int64)
    ijk = torch.empty((3, N_MAX), device=dev, dtype=torch.int16)
    ijk[0, :m] = (idx % side).to(torch.int16)
    ijk[1, :m] = ((idx // side) % side).to(torch.int16)
    ijk[2, :m] = (idx // (side * side)).to(torch.int16)
    del idx
    ijk[:, m:] = torch.from_numpy(np.ascontiguousarray(shell.ijk).view(np.int16)).to(dev)
    level = torch.full((N_MAX,), SLAB_LEVEL, device=dev, dtype=torch.uint8)
    level[m:] = torch.from_numpy(shell.level).to(dev)
    dens = torch.ones((8, N_MAX), device=dev, dtype=torch.float32)
    dens[:, m:] = to_dev(shell.density, dev)
    sh = torch.zeros((3, N_MAX), device=dev, dtype=torch.float32)
    sh[:, m:] = to_dev(shell.sh, dev)
    return ijk, level, dens, sh, shell, m


def test_max_voxel_count(ctx):
    import torch
    import paper_2511_02510_amd as lv
    dev = ctx.device
    say(f"n = 2^28 - 1 = {N_MAX} voxels: slab behind the camera, shell with the top ids")
    ijk, level, dens, sh, shell, m = _slab_and_shell(dev)
    vox = lv.Voxels(ijk, level, dens, sh, shell.root_min, shell.root_size, shell.sh_degree)
    # looking up the z axis, 1 degree off it, from just above the slab: every
    # slab corner lies behind the camera
    o = (0.013, 0.021, -0.96)
    tgt = (0.013 + np.tan(np.radians(1.0)) * 0.6, 0.021 + np.tan(np.radians(1.0)) * 0.8, 0.04)
    cams = [look_at(o, 64, 48, target=tgt)]
    frame = lv.Frame(cams, dev)
    P = frame.P
    r = lv.Renderer(ctx, vox, frame, lv.settings(tile=16, chunk=64))
    rgb, depth, alpha = r.new_outputs()
    wmax = torch.zeros(N_MAX, device=dev)
    r.forward(rgb, depth, alpha, wmax)
    g_rgb, g_depth, g_alpha = random_grads(np.random.default_rng(162), P)
    dd, dsh = torch.empty_like(dens), torch.empty_like(sh)
    r.backward(to_dev(g_rgb, dev), to_dev(g_depth, dev), to_dev(g_alpha, dev), dd, dsh)
    torch.cuda.synchronize()
    say("  rendered; comparing with the oracle on the shell")

    # every slab voxel culled: zero w_max and zero gradients
    assert int(torch.count_nonzero(wmax[:m])) == 0
    assert int(torch.count_nonzero(dd[:, :m])) == 0 and int(torch.count_nonzero(dsh[:, :m])) == 0

    ref = oracle.render(shell, cams)
    got = dict(rgb=rgb.cpu().numpy().astype(np.float64),
               depth=depth.cpu().numpy().astype(np.float64),
               alpha=alpha.cpu().numpy().astype(np.float64))
    check_images(got, ref)
    assert float(ref["alpha"].max()) > 0.3
    wm = wmax[m:].cpu().numpy().astype(np.float64)
    assert np.abs(wm - ref["wmax"]).max() <= WMAX_TOL
    dd_ref, dsh_ref = oracle.backward(shell, cams, g_rgb, g_depth, g_alpha)
    e1 = rel_l2(dd[:, m:].cpu().numpy().astype(np.float64), dd_ref)
    e2 = rel_l2(dsh[:, m:].cpu().numpy().astype(np.float64), dsh_ref)
    say(f"  gradient rel-L2 density {e1:.2e} sh {e2:.2e}")
    assert e1 <= GRAD_TOL and e2 <= GRAD_TOL

    # keys: the shell's records and tile lists with ids shifted by m
    b = lv.export_bins(ctx, vox, frame, r.st, r.saved)
    vis, rect, code = oracle.project_keys(shell, cams)
    assert not b["vis"][0, :m].any()
    assert np.array_equal(b["vis"][:, m:], vis)
    on = vis == 1
    assert np.array_equal(b["rects"][:, m:][on], rect[on])
    assert np.array_equal(b["codes"][:, m:][on], code[on])
    start, ids, _ = oracle.tile_lists(cams, vis, rect, code, 16)
    assert np.array_equal(b["tile_start"], start)
    assert np.array_equal(b["ids"], ids + m)
    say(f"  {int(start[-1])} pairs, ids in tile lists {int(b['ids'].min())} .. "
        f"{int(b['ids'].max())} (largest possible {N_MAX - 1})")
    assert int(b["ids"].min()) >= m
