"""Pins of the grid-point storage oracle: the number of shared points of full
grids and of a coarse/fine junction by counting, the identity case against the
dense layout, and the chain rule through the gather and the activation against
central finite differences of the FP64 renderer."""
import numpy as np
import pytest

import oracle
from oracle import grid as ogrid
import synth
from synth.scenes import Scene, look_at


def test_full_grids_share_corners():
    # a full g^3 grid has (g + 1)^3 corner points; every interior point is
    # read by 8 voxels, and neighbours along x share 4 points
    for lvl in (1, 2, 3):
        sc = synth.make_scene_grid(np.random.default_rng(lvl), res_level=lvl, sh_degree=0)
        idx, ng = synth.grid_points(sc)
        g = 1 << lvl
        assert ng == (g + 1) ** 3
        assert np.bincount(idx.ravel()).max() == (8 if g > 1 else 1)
        pos = {tuple(sc.ijk[:, v]): v for v in range(sc.n)}
        if g > 1:
            a, b = pos[(0, 0, 0)], pos[(1, 0, 0)]
            assert set(idx[[1, 3, 5, 7], a]) == set(idx[[0, 2, 4, 6], b])


def test_coarse_fine_junction_points():
    # one level-1 cell next to its 8 level-2 refinements: 27 points of the
    # fine block + the coarse cell's 8 corners, 4 of them shared = 31
    ijk = [(1, 0, 0)] + [(x, y, z) for z in (0, 1) for y in (0, 1) for x in (0, 1)]
    lev = [1] + [2] * 8
    sc = Scene(root_min=np.array([-1, -1, -1], np.float32), root_size=2.0,
               ijk=np.array(ijk, np.uint16).T.copy(), level=np.array(lev, np.uint8),
               density=np.ones((8, 9), np.float32), sh=np.ones((3, 9), np.float32), sh_degree=0)
    _, ng = synth.grid_points(sc)
    assert ng == 31


def _small_problem(act, seed):
    rng = np.random.default_rng(seed)
    scene = synth.make_scene_shell(rng, 400, 3, 6, sh_degree=1, clutter_frac=0.3)
    idx, ng = synth.grid_points(scene)
    raw = rng.normal(0.3 if act == ogrid.ACT_NONE else -0.5, 0.4, ng)
    if act == ogrid.ACT_NONE:
        raw = np.abs(raw) + 0.05          # non-negative: no clamp of the optical depth
    cams = [look_at((1.9, 0.8, 1.3), 28, 21), look_at((-0.9, 1.4, -1.7), 24, 20)]
    return scene, idx, raw, cams


def test_identity_storage_equals_dense():
    rng = np.random.default_rng(0)
    scene = synth.make_scene_shell(rng, 300, 3, 6, sh_degree=0)
    n = scene.n
    idx = (np.arange(8)[:, None] * n + np.arange(n)[None, :]).astype(np.int32)
    raw = scene.density.astype(np.float64).ravel()
    assert np.array_equal(ogrid.corner_values(raw, idx, ogrid.ACT_NONE), scene.density.astype(np.float64))
    d = rng.normal(0, 1, (8, n))
    assert np.array_equal(ogrid.grid_gradient(d, raw, idx, ogrid.ACT_NONE), d.ravel())
    idx_bad = idx.copy()
    idx_bad[3, 5], idx_bad[0, 7] = -1, 8 * n
    cv = ogrid.corner_values(raw, idx_bad, ogrid.ACT_SOFTPLUS)
    assert cv[3, 5] == 0.0 and cv[0, 7] == 0.0


@pytest.mark.parametrize("act", [ogrid.ACT_NONE, ogrid.ACT_SOFTPLUS, ogrid.ACT_EXP])
def test_grid_gradient_matches_central_differences(act):
    scene, idx, raw, cams = _small_problem(act, 10 + act)
    P = sum(c.npix for c in cams)
    rng = np.random.default_rng(20 + act)
    g_rgb = rng.normal(0, 1, 3 * P)
    g_alpha = rng.normal(0, 1, P)

    def loss(r):
        out = oracle.render(ogrid.with_corners(scene, ogrid.corner_values(r, idx, act)), cams)
        return float(g_rgb @ out["rgb"] + g_alpha @ out["alpha"])

    dc, _ = oracle.backward(ogrid.with_corners(scene, ogrid.corner_values(raw, idx, act)), cams,
                            g_rgb, None, g_alpha)
    d = ogrid.grid_gradient(dc, raw, idx, act)
    shared = np.bincount(idx.ravel(), minlength=raw.shape[0])
    cand = np.nonzero((np.abs(d) > 1e-3) & (shared > 1))[0]
    assert cand.shape[0] >= 10
    pick = rng.choice(cand, size=min(24, cand.shape[0]), replace=False)
    h = 1e-5
    for gidx in pick:
        rp, rm = raw.copy(), raw.copy()
        rp[gidx] += h
        rm[gidx] -= h
        fd = (loss(rp) - loss(rm)) / (2 * h)
        assert abs(fd - d[gidx]) <= 2e-5 * max(1.0, abs(d[gidx])), (gidx, fd, d[gidx])
