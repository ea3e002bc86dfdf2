"""Pins of the subdivision oracle (Sec. IV-D, eq. 13-16, and the 8-way split):
the children reproduce the parent's trilinear density field, a refined scene
renders the same colour and opacity through the FP64 renderer, the children
tile the parent, budgeted selection against sequential brute force, and the
eligibility and far-bias rules."""
import numpy as np

import oracle
from oracle import quantile, split
import synth
from synth.scenes import look_at

f32 = np.float32


def _trilinear(s, u):
    # s [8] corner values (corner c = x + 2y + 4z), u [..., 3] in [0, 1]
    x, y, z = u[..., 0], u[..., 1], u[..., 2]
    out = 0.0
    for c in range(8):
        wx = x if c & 1 else 1 - x
        wy = y if c & 2 else 1 - y
        wz = z if c & 4 else 1 - z
        out = out + s[c] * wx * wy * wz
    return out


def test_children_reproduce_the_parent_field():
    rng = np.random.default_rng(0)
    dens = rng.normal(0, 2, (8, 50)).astype(f32)
    kids = split.child_densities(dens)
    u = rng.uniform(0, 1, (400, 3))
    for j in range(dens.shape[1]):
        for ch in range(8):
            b = np.array([(ch >> a) & 1 for a in range(3)], np.float64)
            parent_u = (b + u) / 2.0
            want = _trilinear(dens[:, j].astype(np.float64), parent_u)
            got = _trilinear(kids[ch, :, j].astype(np.float64), u)
            assert np.abs(got - want).max() <= 4e-6 * (1 + np.abs(dens[:, j]).max())


def test_children_tile_the_parent():
    rng = np.random.default_rng(1)
    scene = synth.make_scene_shell(rng, 500, 3, 7, sh_degree=1)
    sel = (rng.random(scene.n) < 0.3).astype(np.uint8)
    ref = split.apply_split(scene, sel)
    assert ref.n == scene.n + 7 * int(sel.sum())
    pos = 0
    for v in range(scene.n):
        e = scene.root_size * 2.0 ** -int(scene.level[v])
        lo = scene.root_min + scene.ijk[:, v] * e
        if not sel[v]:
            assert np.array_equal(ref.ijk[:, pos], scene.ijk[:, v]) and ref.level[pos] == scene.level[v]
            assert np.array_equal(ref.density[:, pos], scene.density[:, v])
            pos += 1
            continue
        boxes = set()
        for c in range(8):
            k = pos + c
            assert ref.level[k] == scene.level[v] + 1
            ek = scene.root_size * 2.0 ** -int(ref.level[k])
            clo = scene.root_min + ref.ijk[:, k] * ek
            off = np.round((clo - lo) / ek).astype(int)
            assert np.allclose(clo, lo + off * ek) and np.all((off >= 0) & (off <= 1))
            boxes.add(tuple(off))
            assert np.array_equal(ref.sh[:, k], scene.sh[:, v])
        assert len(boxes) == 8
        pos += 8
    assert pos == ref.n


def test_refined_scene_renders_the_same_colour_and_opacity():
    # constant colour per voxel (SH degree 0): the density field is unchanged
    # by the split and the children share the parent's colour, so every ray
    # accumulates the same optical depth through them
    rng = np.random.default_rng(2)
    scene = synth.make_scene_shell(rng, 3000, 4, 7, sh_degree=0, clutter_frac=0.2)
    cams = [look_at((1.9, 0.7, 1.2), 48, 36), look_at((-0.6, 1.1, -2.1), 40, 30)]
    sel = (rng.random(scene.n) < 0.4).astype(np.uint8)
    ref = split.apply_split(scene, sel)
    a = oracle.render(scene, cams)
    b = oracle.render(ref, cams)
    assert np.abs(a["alpha"]).max() > 0.3
    assert np.abs(a["rgb"] - b["rgb"]).max() <= 1e-5
    assert np.abs(a["alpha"] - b["alpha"]).max() <= 1e-5


def _sequential_pick(cand, prio, k):
    left = [i for i in range(cand.shape[0]) if cand[i]]
    out = np.zeros(cand.shape[0], np.uint8)
    for _ in range(min(k, len(left))):
        best = left[0]
        for i in left[1:]:
            if float(prio[i]) > float(prio[best]) or (float(prio[i]) == float(prio[best]) and i < best):
                best = i
        out[best] = 1
        left.remove(best)
    return out


def test_budgeted_selection_matches_sequential_picking():
    rng = np.random.default_rng(3)
    scene = synth.make_scene_shell(rng, 600, 3, 8, sh_degree=0, clutter_frac=0.3)
    cams = [look_at((1.7, 0.9, 1.5), 64, 48), look_at((0.4, -1.8, 1.6), 80, 60)]
    z5, z95 = split.footprint_range(scene, cams)
    for trial in range(12):
        score = rng.choice(np.array([0.0, 0.5, 1.0, 2.0, 0.25], f32), scene.n)   # ties
        k = int(rng.integers(0, 200))
        got, prio, elig = split.select(scene, cams, score, z5, z95, kappa=0.3, beta=0.2, max_splits=k)
        want = _sequential_pick(elig & (prio > 0), prio, k)
        assert np.array_equal(got, want), trial


def test_eligibility_rules():
    rng = np.random.default_rng(4)
    scene = synth.make_scene_shell(rng, 2000, 8, 12, sh_degree=0, clutter_frac=0.2)
    cams = [look_at((0.0, 0.1, 0.2), 64, 48, target=(0.0, 0.1, -1.0))]   # inside: some unseen
    z5, z95 = split.footprint_range(scene, cams)
    delta = quantile.depth_proxy(scene, cams)
    score = np.ones(scene.n, f32)
    s, prio, elig = split.select(scene, cams, score, z5, z95, kappa=1e-6, max_splits=scene.n)
    assert not np.any(elig & (scene.level == 12))          # the finest level never splits
    assert not np.any(elig & ~np.isfinite(delta))          # no footprint, no split
    assert np.array_equal(s.astype(bool), elig)
    assert (scene.level == 12).any() and (~np.isfinite(delta)).any() and elig.any()
    s2, _, elig2 = split.select(scene, cams, score, z5, z95, kappa=1e9, max_splits=scene.n)
    assert not elig2.any() and not s2.any()                 # eq. 13 with a huge kappa
    h = 0.5 * scene.root_size * 2.0 ** -scene.level.astype(np.float64)
    assert np.all(h[elig] > 1e-6 * delta[elig])


def test_far_bias_prefers_far_voxels():
    # equal usefulness: the far bias (eq. 15-16) decides, farther first
    rng = np.random.default_rng(5)
    scene = synth.make_scene_shell(rng, 3000, 4, 8, sh_degree=0, clutter_frac=0.5)
    cams = [look_at((2.2, 0.5, 1.0), 64, 48)]
    z5, z95 = split.footprint_range(scene, cams)
    delta = quantile.depth_proxy(scene, cams)
    zt = split.normalised_depth(delta, z5, z95)
    score = np.ones(scene.n, f32)
    s, prio, elig = split.select(scene, cams, score, z5, z95, kappa=0.05, beta=0.3, max_splits=100)
    assert s.sum() == 100
    assert zt[s == 1].min() >= zt[elig & (s == 0)].max()
    assert prio[s == 1].min() >= prio[elig & (s == 0)].max()
    # without the bias every eligible voxel ties and the lowest indices win
    s0, _, _ = split.select(scene, cams, score, z5, z95, kappa=0.05, beta=0.0, max_splits=100)
    assert np.array_equal(np.nonzero(s0)[0], np.nonzero(elig)[0][:100])
