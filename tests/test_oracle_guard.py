"""Pins of the pruning-guard oracle (Sec. IV-C, guards i-iii) against closed
forms, a worked sequence, brute-force removal and the unguarded quantile
decision of eq. 12."""
import math

import numpy as np

from oracle import guard, quantile
import synth
from synth.scenes import look_at

f32 = np.float32


def _scene_and_cams(n=3000, seed=11):
    rng = np.random.default_rng(seed)
    scene = synth.make_scene_shell(rng, n, 4, 8, sh_degree=0, clutter_frac=0.2)
    cams = [look_at((2.1, 0.6, 1.3), 64, 48), look_at((-0.5, 1.2, -2.2), 80, 60)]
    return scene, cams


def test_ema_closed_form():
    # x held at 1 (or 0) for t steps: m_t = 1 - (1-a)^t (1 - m_0)  (or m_0 (1-a)^t)
    rng = np.random.default_rng(0)
    m0 = rng.uniform(0, 1, 1000).astype(f32)
    for a in (0.05, 0.3, 0.9):
        up, down = m0.copy(), m0.copy()
        for t in range(1, 25):
            up = guard.ema_update(up, np.ones_like(m0), a)
            down = guard.ema_update(down, np.zeros_like(m0), a)
            keep = (1.0 - float(f32(a))) ** t
            assert np.abs(up - (1.0 - keep * (1.0 - m0.astype(np.float64)))).max() < 4e-6 * t
            assert np.abs(down - m0.astype(np.float64) * keep).max() < 4e-6 * t
        assert up.dtype == f32 and np.all(up <= 1.0) and np.all(down >= 0.0)


def test_hysteresis_worked_sequence():
    # alpha = 1/2, thresholds 0.3 / 0.7, start in with m = 1; the inside
    # score runs 0, 0, 1, 1, 0.  By hand: m = 1/2 (between: stays in),
    # 1/4 (< 0.3: out), 5/8 (between: stays out), 13/16 (> 0.7: in),
    # 13/32 (between: stays in).  All values are dyadic, so exact in binary32.
    m = np.array([1.0], f32)
    s = np.array([1], np.uint8)
    got_m, got_s = [], []
    for x in (0, 0, 1, 1, 0):
        m = guard.ema_update(m, np.array([x], f32), 0.5)
        s = guard.hysteresis(m, s, 0.3, 0.7)
        got_m.append(float(m[0]))
        got_s.append(int(s[0]))
    assert got_m == [0.5, 0.25, 0.625, 0.8125, 0.40625]
    assert got_s == [1, 0, 0, 1, 1]


def test_order_key_is_the_binary32_order():
    v = np.array([0.5, -0.0, 0.0, -1.0, np.inf, 1e-38, 3.0, -np.inf, 2.5e-3], f32)
    k = guard.order_key(v)
    srt = v[np.argsort(k, kind="stable")]
    assert np.all(np.diff(srt.astype(np.float64)) >= 0)
    assert np.signbit(v[np.argsort(k)[2]]) and not np.signbit(v[np.argsort(k)[3]])   # -0 then +0


def _sequential_cap(cand, m, cap_frac):
    # remove, one at a time, the remaining candidate with the smallest (m, index)
    n = cand.shape[0]
    cap = int(math.floor(cap_frac * n))
    left = [i for i in range(n) if cand[i]]
    prune = np.zeros(n, np.uint8)
    for _ in range(min(cap, len(left))):
        best = left[0]
        for i in left[1:]:
            if float(m[i]) < float(m[best]) or (float(m[i]) == float(m[best]) and i < best):
                best = i
        prune[best] = 1
        left.remove(best)
    return prune


def test_cap_matches_sequential_removal():
    rng = np.random.default_rng(3)
    for trial in range(30):
        n = int(rng.integers(1, 300))
        cand = rng.random(n) < rng.uniform(0.05, 0.9)
        m = rng.choice(np.array([0.0, 0.125, 0.25, 0.2, 0.29], f32), n)   # many ties
        for frac in (0.0, 0.01, 0.1, 0.5, 1.0):
            got = guard.capped_prune(cand, m, frac)
            assert np.array_equal(got, _sequential_cap(cand, m, frac)), (trial, frac)
            assert got.sum() == min(int(math.floor(frac * n)), int(cand.sum()))


def test_guard_with_neutral_settings_is_the_quantile_decision():
    # alpha = 1 (m = x), one threshold 0.5, no halo, no cap: prune exactly the
    # voxels with w_max <= tau_bin (eq. 12)
    scene, cams = _scene_and_cams()
    rng = np.random.default_rng(5)
    wmax = (rng.uniform(0, 1, scene.n) ** 3).astype(f32)
    wmax[rng.random(scene.n) < 0.1] = 0.0
    bins, _, _ = quantile.depth_bins(quantile.depth_proxy(scene, cams), 16)
    tau, qprune = quantile.quantile_cutoffs(wmax, bins, 16, 0.1)
    prune, m, s = guard.guard_step(scene, cams, wmax, bins, tau, np.ones(scene.n, f32),
                                   np.ones(scene.n, np.uint8), alpha=1.0, m_low=0.5, m_high=0.5,
                                   rho=0.0, w_keep=2.0, cap_frac=1.0)
    assert np.array_equal(prune, qprune)
    assert np.array_equal(s, 1 - qprune)


def test_halo_and_cap_invariants_over_steps():
    scene, cams = _scene_and_cams()
    rng = np.random.default_rng(7)
    delta = quantile.depth_proxy(scene, cams)
    h = (f32(0.5) * np.ldexp(f32(scene.root_size), -scene.level.astype(np.int32))).astype(f32)
    m = np.ones(scene.n, f32)
    s = np.ones(scene.n, np.uint8)
    bins, _, _ = quantile.depth_bins(delta, 8)
    total = 0
    for step in range(6):
        wmax = (rng.uniform(0, 1, scene.n) ** 4).astype(f32)
        tau, _ = quantile.quantile_cutoffs(wmax, bins, 8, 0.3)
        prev_s = s
        prune, m, s = guard.guard_step(scene, cams, wmax, bins, tau, m, s, alpha=0.4,
                                       m_low=0.35, m_high=0.65, rho=0.6, w_keep=0.8,
                                       cap_frac=0.02)
        small = np.isfinite(delta) & (h < (f32(0.6) * np.where(np.isfinite(delta), delta, 0)))
        assert not np.any(prune & (small | (wmax >= f32(0.8))))        # keep-halo
        assert prune.sum() <= math.floor(0.02 * scene.n)               # per-step cap
        assert np.all(s[prune == 1] == 0)                              # only "out" voxels
        # states change only across the thresholds (hysteresis)
        flip = s != prev_s
        assert np.all((m[flip & (s == 0)] < f32(0.35))) and np.all(m[flip & (s == 1)] > f32(0.65))
        cand_left = (s == 0) & ~(small | (wmax >= f32(0.8))) & (prune == 0)
        if prune.any() and cand_left.any():
            assert guard.order_key(m[prune == 1]).max() <= guard.order_key(m[cand_left]).min()
        total += int(prune.sum())
    assert total > 0


def test_voxels_no_view_sees_in_front_are_not_size_protected():
    # one camera inside the shell: voxels behind it have no footprint
    # (delta = +inf); with rho huge every other voxel is size-protected, so
    # only the unseen ones can be pruned
    rng = np.random.default_rng(9)
    scene = synth.make_scene_shell(rng, 2000, 4, 7, sh_degree=0)
    cams = [look_at((0.0, 0.1, 0.2), 40, 30, target=(0.0, 0.1, -1.0))]
    delta = quantile.depth_proxy(scene, cams)
    unseen = ~np.isfinite(delta)
    assert unseen.sum() > 100 and (~unseen).sum() > 100
    bins, _, _ = quantile.depth_bins(delta, 4)
    wmax = np.zeros(scene.n, f32)
    tau = np.full(4, 0.5, f32)
    prune, _, s = guard.guard_step(scene, cams, wmax, bins, tau, np.zeros(scene.n, f32),
                                   np.zeros(scene.n, np.uint8), alpha=0.5, rho=1e30,
                                   w_keep=2.0, cap_frac=1.0)
    assert np.all(s == 0)
    assert np.array_equal(prune.astype(bool), unseen)
