"""Properties of the seeded input generators (CPU)."""
import numpy as np

import synth


def _leaf_keys(sc):
    return [(int(l), int(sc.ijk[0, v]), int(sc.ijk[1, v]), int(sc.ijk[2, v]))
            for v, l in enumerate(sc.level)]


def _assert_no_overlap(sc):
    keys = _leaf_keys(sc)
    s = set(keys)
    assert len(s) == len(keys)                       # no duplicates
    for (l, x, y, z) in keys:
        for up in range(1, l + 1):                   # no leaf inside another
            assert (l - up, x >> up, y >> up, z >> up) not in s


def test_shell_scene_is_an_overlap_free_octree_with_level_law():
    rng = np.random.default_rng(0)
    sc = synth.make_scene_shell(rng, 20000, 6, 9, sh_degree=3)
    assert sc.n == 20000
    _assert_no_overlap(sc)
    h = np.bincount(sc.level, minlength=10)[6:10].astype(np.float64)
    p = np.exp2(np.arange(6, 10))
    assert np.allclose(h / h.sum(), p / p.sum(), atol=1e-3)
    e = sc.root_size * np.exp2(-sc.level.astype(np.float64))
    c = sc.root_min[:, None] + (sc.ijk + 0.5) * e
    r = np.linalg.norm(c, axis=0)
    assert np.all(r > 0.75 - 0.2) and np.all(r < 0.85 + 0.2)
    assert sc.density.dtype == np.float32 and np.all(sc.density > 0)
    assert sc.sh.shape == (48, 20000)
    assert np.all((sc.sh[0:3] >= 0) & (sc.sh[0:3] <= 1))


def test_clutter_and_determinism():
    a = synth.make_scene_shell(np.random.default_rng(4), 5000, 5, 8, clutter_frac=0.1)
    b = synth.make_scene_shell(np.random.default_rng(4), 5000, 5, 8, clutter_frac=0.1)
    assert np.array_equal(a.ijk, b.ijk) and np.array_equal(a.density, b.density)
    _assert_no_overlap(a)


def test_named_small_configs():
    sc, cams, tg = synth.make_config("grid4k")
    assert sc.n == 4096 and sc.sh_degree == 0 and len(cams) == 1
    assert cams[0].width == 64 and tg[0].shape == (3, 64, 64)
    R = cams[0].R.astype(np.float64)
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-6)
    # camera looks at the origin
    f = -cams[0].o / np.linalg.norm(cams[0].o)
    assert np.allclose(R[2], f, atol=1e-6)
    ring = synth.make_cameras_ring(np.random.default_rng(0), 8)
    assert len(ring) == 8 and all((c.width, c.height) in synth.scenes.RING_RESOLUTIONS for c in ring)
    hemi = synth.make_cameras_hemisphere()
    assert len(hemi) == 16 and all(c.o[1] > 0 for c in hemi)


def test_leaves_are_stored_in_octree_order():
    # depth-first order: a leaf's minimum corner at the finest level, bits
    # interleaved, never decreases; every ancestor's leaves are contiguous
    sc = synth.make_scene_shell(np.random.default_rng(9), 3000, 4, 7)
    fine = [(sc.ijk[a].astype(np.int64) << (synth.scenes.L_MAX - sc.level.astype(np.int64)))
            for a in range(3)]
    def morton(v):
        k = 0
        for b in range(synth.scenes.L_MAX):
            for a in range(3):
                k |= int((fine[a][v] >> b) & 1) << (3 * b + a)
        return k
    keys = [morton(v) for v in range(sc.n)]
    assert all(keys[i] < keys[i + 1] for i in range(sc.n - 1))
    # leaves under one level-2 cell form one run
    top = [tuple(int(fine[a][v] >> (synth.scenes.L_MAX - 2)) for a in range(3)) for v in range(sc.n)]
    seen, prev = set(), None
    for t in top:
        if t != prev:
            assert t not in seen
            seen.add(t)
            prev = t
    g, _, _ = synth.make_config("grid4k")
    assert g.ijk[:, 1].tolist() == [1, 0, 0] and g.ijk[:, 2].tolist() == [0, 1, 0]


def test_layered_scene_of_the_pruning_study():
    """The two shells of the pruning study form one overlap-free leaf set in
    octree order; the tag marks the outer shell's leaves and the inner
    shell is the denser one."""
    from paper_2511_02510_amd.train import layered_scene
    sc, outer, inner_sc, outer_sc = layered_scene()
    assert sc.n == inner_sc.n + outer_sc.n == 50000 and int(outer.sum()) == outer_sc.n
    _assert_no_overlap(sc)
    e = sc.root_size * np.exp2(-sc.level.astype(np.float64))
    r = np.linalg.norm(sc.root_min[:, None] + (sc.ijk + 0.5) * e, axis=0)
    assert r[~outer].max() < r[outer].min()
    assert np.median(sc.density[:, ~outer]) > 10 * np.median(sc.density[:, outer])
    order = synth.scenes.octree_order(sc.ijk, sc.level)
    assert np.array_equal(order, np.arange(sc.n))
