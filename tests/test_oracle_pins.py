"""Pins of the FP64 oracle against what the paper and mathematics fix
(closed forms, invariants, brute-force integration, library routines).
CPU only."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import brute, loss, quantile
import synth
from synth.scenes import Camera, Scene, look_at

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def one_voxel_scene(sigma, colour, root_min=(-0.5, -0.5, -0.5), size=1.0, level=0, ijk=(0, 0, 0)):
    dens = np.asarray(sigma, np.float32).reshape(8, 1) if np.ndim(sigma) else \
        np.full((8, 1), sigma, np.float32)
    return Scene(root_min=np.array(root_min, np.float32), root_size=size,
                 ijk=np.array(ijk, np.uint16).reshape(3, 1), level=np.array([level], np.uint8),
                 density=dens, sh=np.asarray(colour, np.float32).reshape(3, 1), sh_degree=0)


def axis_camera(o, target, res=65):
    # odd resolution: the central pixel's ray is exactly the optical axis
    return look_at(o, res, res, target=target)


def centre_dir(cam, px, py):
    dc = np.array([(px + 0.5 - cam.cx) / cam.fx, (py + 0.5 - cam.cy) / cam.fy, 1.0])
    d = np.asarray(cam.R, np.float64).T @ dc
    return d / np.linalg.norm(d)


# -------------------------------------------------------------- T1 closed form
def test_single_voxel_constant_density_closed_form():
    sigma, col = float(np.float32(1.3)), tuple(float(np.float32(c)) for c in (0.2, 0.6, 0.9))
    sc = one_voxel_scene(sigma, col)
    cam = axis_camera((0.0, 0.0, -3.0), (0.0, 0.0, 0.0))
    out = oracle.render(sc, [cam])
    A = out["alpha"].reshape(65, 65)
    rgb = out["views"][0]
    checked = 0
    for py in range(65):
        for px in range(65):
            d = centre_dir(cam, px, py)
            # rays entering the front face z=-0.5 and leaving the back face z=0.5
            t_in, t_out = 2.5 / d[2], 3.5 / d[2]
            p_in, p_out = cam.o + t_in * d, cam.o + t_out * d
            if max(abs(p_in[0]), abs(p_in[1]), abs(p_out[0]), abs(p_out[1])) >= 0.5:
                continue
            ell = t_out - t_in
            a = -math.expm1(-sigma * ell)
            assert abs(A[py, px] - a) < 1e-12
            for ch in range(3):
                assert abs(rgb[ch, py, px] - a * col[ch]) < 1e-12
            assert abs(out["depth"][py * 65 + px] - a * 0.5 * (t_in + t_out)) < 1e-11
            checked += 1
    assert checked > 100
    # the central ray runs along the axis: chord exactly 1
    assert abs(A[32, 32] - (1 - math.exp(-sigma))) < 1e-14
    # eq. 5 with a single voxel: w_max is the largest opacity over the pixel rays
    assert abs(out["wmax"][0] - A.max()) < 1e-15
    assert 0.0 < out["wmax"][0] <= 1.0


# ------------------------------------------------------------ T2 two voxels
def test_two_stacked_voxels_closed_form():
    g = GOLDEN["two_voxel_stack"]
    f = lambda x: np.float32(x).astype(np.float64)
    s1, s2, c1, c2 = float(f(g["sigma1"])), float(f(g["sigma2"])), f(g["c1"]), f(g["c2"])
    sc = Scene(root_min=np.array([-1, -1, -1], np.float32), root_size=2.0,
               ijk=np.array([[0, 0], [0, 0], [0, 1]], np.uint16),
               level=np.array([1, 1], np.uint8),
               density=np.array([[s1, s2]] * 8, np.float32),
               sh=np.stack([c1, c2], axis=1).astype(np.float32), sh_degree=0)
    cam = axis_camera((-0.5, -0.5, -4.0), (-0.5, -0.5, 0.0))
    out = oracle.render(sc, [cam])
    a1, a2 = 1 - math.exp(-s1), 1 - math.exp(-s2)
    C = a1 * c1 + (1 - a1) * a2 * c2
    A = 1 - (1 - a1) * (1 - a2)
    D = a1 * g["t_mid1"] + (1 - a1) * a2 * g["t_mid2"]
    k = 32 * 65 + 32
    assert np.allclose(out["views"][0][:, 32, 32], C, atol=1e-13, rtol=0)
    assert abs(out["alpha"][k] - A) < 1e-13
    assert abs(out["depth"][k] - D) < 1e-12
    # background enters through the final transmittance
    bg = (0.3, 0.1, 0.7)
    out2 = oracle.render(sc, [cam], bg=bg)
    assert np.allclose(out2["views"][0][:, 32, 32], C + (1 - A) * np.array(bg), atol=1e-13)
    # the front voxel's w_max is its own alpha on the axis (largest over rays)
    assert out["wmax"][0] >= a1 - 1e-15


# ------------------------------------------------------- T3 linear density
def test_linear_density_integrates_to_midpoint_value():
    a0, grad = 1.0, np.array([0.5, -0.25, 0.375])   # dyadic: exact in float32
    corners = []
    for c in range(8):
        x = np.array([-0.5 + (c & 1), -0.5 + ((c >> 1) & 1), -0.5 + ((c >> 2) & 1)])
        corners.append(a0 + grad @ x)
    assert min(corners) > 0
    sc = one_voxel_scene(corners, (1.0, 1.0, 1.0))
    cam = axis_camera((0.0, 0.0, -3.0), (0.0, 0.0, 0.0))
    out = oracle.render(sc, [cam])
    A = out["alpha"].reshape(65, 65)
    n = 0
    for py in range(10, 55, 3):
        for px in range(10, 55, 3):
            d = centre_dir(cam, px, py)
            t_in, t_out = 2.5 / d[2], 3.5 / d[2]
            p_in, p_out = cam.o + t_in * d, cam.o + t_out * d
            if max(abs(p_in[0]), abs(p_in[1]), abs(p_out[0]), abs(p_out[1])) >= 0.5:
                continue
            mid = cam.o + 0.5 * (t_in + t_out) * d
            tau = (t_out - t_in) * (a0 + grad @ mid)
            assert abs(A[py, px] - (-math.expm1(-tau))) < 1e-12
            n += 1
    assert n > 20


# --------------------------------------------------------------- T4 cubic
@pytest.mark.parametrize("corner,key", [(7, "corner7_integral"), (1, "corner1_integral"),
                                        (0, "corner0_integral")])
def test_cubic_corner_weight_along_diagonal(corner, key):
    sig = np.zeros(8)
    sig[corner] = 2.0
    sc = one_voxel_scene(sig, (1.0, 1.0, 1.0))
    u = np.ones(3) / math.sqrt(3.0)
    cam = axis_camera(tuple(-3.0 * u), (0.0, 0.0, 0.0))
    out = oracle.render(sc, [cam])
    a = out["alpha"][32 * 65 + 32]
    tau = -math.log1p(-a)
    ell = math.sqrt(3.0)
    # the float32 camera makes the ray diagonal only to ~1e-7
    assert abs(tau - 2.0 * ell * GOLDEN["diagonal_corner_integrals"][key]) < 2e-6


# ------------------------------------------------------ T5 invariants
def small_shell(n=3000, seed=5, deg=3, lmin=4, lmax=7, clutter=0.0):
    rng = np.random.default_rng(seed)
    return synth.make_scene_shell(rng, n, lmin, lmax, sh_degree=deg, clutter_frac=clutter)


def test_transmittance_and_weight_invariants():
    sc = small_shell()
    cam = synth.make_cameras_single(48, 40)[0]
    out = oracle.render(sc, [cam])
    assert np.all(out["alpha"] >= 0) and np.all(out["alpha"] <= 1)
    assert np.all(out["wmax"] >= 0) and np.all(out["wmax"] <= 1)
    rng = np.random.default_rng(1)
    seen = 0
    for _ in range(60):
        px, py = rng.integers(0, 48), rng.integers(0, 40)
        tr = oracle.trace_pixel(sc, cam, px, py)
        if tr["vid"].shape[0] == 0:
            continue
        seen += 1
        T = np.concatenate([[1.0], tr["T_after"]])
        assert np.all(T >= 0) and np.all(T <= 1)
        assert np.all(np.diff(T) <= 0)                              # never increases
        assert np.all(np.diff(tr["tin"]) > 0)                       # front to back
        assert abs(tr["w"].sum() - (1 - T[-1])) < 1e-12             # sum w = 1 - T_K
        assert abs(out["alpha"][py * 48 + px] - (1 - T[-1])) < 1e-12
        assert np.all(out["wmax"][tr["vid"]] >= tr["w"] - 1e-15)   # eq. 5
    assert seen > 20


# -------------------------------------------------- T6 brute-force integral
def test_brute_force_ray_integral_matches():
    rng = np.random.default_rng(11)
    # a small cluster of mixed-level leaves around the origin
    sc = small_shell(n=40, seed=3, deg=0, lmin=3, lmax=5)
    cam = look_at((0.4, 2.2, 1.3), 33, 33)
    out = oracle.render(sc, [cam])
    hit_px = np.nonzero(out["n_hits"] > 1)[0]
    assert hit_px.shape[0] > 10
    for k in rng.choice(hit_px, size=6, replace=False):
        px, py = k % 33, k // 33
        d = centre_dir(cam, px, py)
        C, A = brute.integrate_ray(sc, cam.o.astype(np.float64), d, t_max=5.0, n_steps=400_000)
        assert abs(A - out["alpha"][k]) < 1e-4
        assert np.max(np.abs(C - out["views"][0][:, py, px])) < 1e-4


# ------------------------------------------------ T7 visibility code order
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_visibility_code_orders_every_ray(seed):
    rng = np.random.default_rng(100 + seed)
    sc = small_shell(n=400, seed=seed, deg=0, lmin=2, lmax=6, clutter=0.5)
    # camera positions outside and inside the root cube
    o = rng.uniform(-2.5, 2.5, 3) if seed != 2 else np.array([0.13, -0.27, 0.31])
    cam = look_at(o, 40, 32, target=tuple(rng.uniform(-0.3, 0.3, 3)))
    vis, rect, code = oracle.project_keys(sc, [cam])
    checked = 0
    for py in range(0, 32, 3):
        for px in range(0, 40, 3):
            tr = oracle.trace_pixel(sc, cam, px, py)
            v = tr["vid"]
            if v.shape[0] < 2:
                continue
            cds = code[0, v]
            assert np.all(np.diff(cds.astype(np.float64)) > 0) or np.all(cds[1:] > cds[:-1])
            # every voxel with a real chord through this pixel is binned over it
            big = (tr["tout"] - tr["tin"]) > 1e-6
            for vv in v[big]:
                assert vis[0, vv] == 1
                x0, x1, y0, y1 = rect[0, vv]
                assert x0 <= px <= x1 and y0 <= py <= y1
            checked += 1
    assert checked > 20


def test_tile_lists_are_sorted_and_complete():
    sc = small_shell(n=2000, seed=9, deg=0)
    cams = synth.make_cameras_single(70, 45)
    vis, rect, code = oracle.project_keys(sc, cams)
    start, ids, keys = oracle.tile_lists(cams, vis, rect, code, 16)
    assert np.all(np.diff(keys.astype(np.float64)) >= 0)
    assert start[-1] == ids.shape[0]
    # brute: count of (record, tile) overlaps equals the number of pairs
    r = rect[0][vis[0] == 1]
    n = ((r[:, 1] // 16 - r[:, 0] // 16 + 1) * (r[:, 3] // 16 - r[:, 2] // 16 + 1)).sum()
    assert n == ids.shape[0]


# ------------------------------------------------------------------- T8 FD
def _loss_of(sc, cams, targets, weights, a_depth, b_alpha):
    out = oracle.render(sc, cams)
    L = 0.0
    for v, c in enumerate(cams):
        l, _ = loss.l1_loss_grad(out["views"][v], targets[v], weights[v])
        L += l
    L += float(a_depth @ out["depth"]) + float(b_alpha @ out["alpha"])
    return L, out


def test_analytic_gradient_matches_central_differences():
    rng = np.random.default_rng(7)
    sc = small_shell(n=1500, seed=4, deg=3, lmin=4, lmax=6)
    cams = [look_at((1.2, 0.9, 2.0), 40, 30), look_at((-2.0, 0.5, 1.0), 36, 28)]
    targets = [synth.make_target(rng, c.width, c.height) for c in cams]
    weights = [loss.lf_weight(t, gamma=0.5, form=1) for t in targets]
    P = sum(c.npix for c in cams)
    a_depth = rng.normal(0, 1e-3, P)
    b_alpha = rng.normal(0, 1e-2, P)
    L0, out = _loss_of(sc, cams, targets, weights, a_depth, b_alpha)
    g_rgb = oracle.join_views([loss.l1_loss_grad(out["views"][v], targets[v], weights[v])[1]
                               for v in range(len(cams))])
    dd, dsh = oracle.backward(sc, cams, g_rgb, a_depth, b_alpha)
    resid_sign = [np.sign(out["views"][v] - targets[v]) for v in range(len(cams))]
    raw0, _ = oracle.voxel_colours(sc, cams)
    hit = np.nonzero(out["wmax"] > 1e-3)[0]
    h = 1e-3
    fd, an = [], []
    tries = 0
    while len(fd) < 64 and tries < 400:
        tries += 1
        v = int(rng.choice(hit))
        if len(fd) < 32:
            arr, row = "density", int(rng.integers(0, 8))
        else:
            arr, row = "sh", int(rng.integers(0, 48))
        vals = []
        ok = True
        for sgn in (+1, -1):
            s2 = synth.scene_subset(sc, np.arange(sc.n))
            getattr(s2, arr)[row, v] += np.float32(sgn * h)
            Lp, o2 = _loss_of(s2, cams, targets, weights, a_depth, b_alpha)
            for vv in range(len(cams)):
                if np.any(np.sign(o2["views"][vv] - targets[vv]) != resid_sign[vv]):
                    ok = False
            raw2, _ = oracle.voxel_colours(s2, cams)
            if np.any((raw2[:, v] > 0) != (raw0[:, v] > 0)):
                ok = False
            vals.append(Lp)
        if not ok:
            continue
        # the perturbation actually applied is the float32 rounding of +-h
        hp = float(np.float32(getattr(sc, arr)[row, v] + np.float32(h)) - getattr(sc, arr)[row, v])
        hm = float(getattr(sc, arr)[row, v] - np.float32(getattr(sc, arr)[row, v] - np.float32(h)))
        fd.append((vals[0] - vals[1]) / (hp + hm))
        an.append(dd[row, v] if arr == "density" else dsh[row, v])
    assert len(fd) == 64
    fd, an = np.array(fd), np.array(an)
    rel = np.linalg.norm(fd - an) / np.linalg.norm(an)
    assert rel < 1e-4, rel


# ---------------------------------------------------------------- T9 SH
def test_sh_basis_orthonormal_and_addition_theorem():
    xg, wg = np.polynomial.legendre.leggauss(24)
    phis = (np.arange(48) + 0.5) * 2 * math.pi / 48
    ct, ph = np.meshgrid(xg, phis, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=-1).reshape(-1, 3)
    wq = (wg[:, None] * np.full(48, 2 * math.pi / 48)[None, :]).ravel()
    Y = oracle.sh_basis(dirs, 3)
    G = (Y * wq[:, None]).T @ Y
    assert np.max(np.abs(G - np.eye(16))) < 1e-12
    rng = np.random.default_rng(0)
    d = rng.normal(size=(50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = oracle.sh_basis(d, 3)
    for l in range(4):
        s = (Y[:, l * l:(l + 1) * (l + 1)] ** 2).sum(axis=1)
        assert np.allclose(s, (2 * l + 1) / (4 * math.pi), atol=1e-13)
    # degree 1 is a rotation of the coordinates: |Y_1(d)| is sqrt(3/4pi)|d|
    assert np.allclose(np.abs(Y[:, 2]), math.sqrt(3 / (4 * math.pi)) * np.abs(d[:, 2]))


def test_degree_zero_colour_is_the_constant_term():
    sc = small_shell(n=300, seed=1, deg=0, lmin=3, lmax=5)
    cams = synth.make_cameras_single(16, 16)
    raw, col = oracle.voxel_colours(sc, cams)
    assert np.allclose(raw[0], sc.sh[0:3].T.astype(np.float64))


# ----------------------------------------------------------- T10 loss pins
def test_inverse_sobel_weight_pins():
    from scipy import ndimage
    rng = np.random.default_rng(3)
    tgt = synth.make_target(rng, 50, 37)
    grey = tgt.astype(np.float64).mean(0)
    g_ref = np.hypot(ndimage.sobel(grey, axis=1, mode="nearest"),
                     ndimage.sobel(grey, axis=0, mode="nearest"))
    assert np.allclose(loss.sobel_magnitude(grey), g_ref, atol=1e-12)
    assert loss.nearest_rank(g_ref, 0.99) == np.quantile(g_ref, 0.99, method="inverted_cdf")
    for form in (0, 1):
        w0 = loss.lf_weight(tgt, gamma=0.0, form=form)
        assert np.allclose(w0, 1.0)                                   # gamma = 0
        w = loss.lf_weight(tgt, gamma=0.6, form=form)
        assert abs(w.mean() - 1.0) < 1e-12                            # eq. 8
        flat = g_ref <= np.quantile(g_ref, 0.1, method="inverted_cdf")
        edge = g_ref >= np.quantile(g_ref, 0.99, method="inverted_cdf")
        assert w[flat].min() > w[edge].max()                          # flats up-weighted
    # eq. 10 with gamma = 0 is the plain L1 loss
    rgb = rng.uniform(0, 1, tgt.shape)
    l, gr = loss.l1_loss_grad(rgb, tgt, loss.lf_weight(tgt, 0.0))
    assert abs(l - np.abs(rgb - tgt).mean()) < 1e-12
    # gradient of the plain L1 is sign/(3 |P|), checked numerically on a few pixels
    for (c, y, x) in [(0, 3, 4), (2, 20, 30), (1, 36, 49)]:
        r2 = rgb.copy()
        r2[c, y, x] += 1e-6
        l2, _ = loss.l1_loss_grad(r2, tgt, loss.lf_weight(tgt, 0.0))
        assert abs((l2 - l) / 1e-6 - gr[c, y, x]) < 1e-6


def test_eq7_weight_extremes():
    tgt = np.zeros((3, 20, 20), np.float32)
    tgt[:, :, 10:] = 1.0                                              # one vertical edge
    w = loss.lf_weight(tgt, gamma=1.0, form=0, eps=1e-3)
    raw = np.where(np.abs(np.arange(20) - 9.5) < 1, 1e-3, 1.0 + 1e-3)  # s = 1 on the edge
    raw = np.broadcast_to(raw, (20, 20))
    assert np.allclose(w, raw / raw.mean())


# ------------------------------------------------------- T11 quantile
def test_bin_quantile_equals_inverted_cdf():
    rng = np.random.default_rng(5)
    wmax = rng.uniform(0, 1, 5000).astype(np.float32)
    wmax[:200] = 0.0                                                   # ties at zero
    bins = rng.integers(0, 16, 5000)
    bins[bins == 7] = 8                                                # an empty bin
    tau, prune = quantile.quantile_cutoffs(wmax, bins, 16, 0.1)
    for b in range(16):
        x = wmax[bins == b]
        if x.shape[0] == 0:
            assert tau[b] == -np.inf
            continue
        assert tau[b] == np.quantile(x, 0.1, method="inverted_cdf")
        assert np.all(prune[bins == b] == (x <= tau[b]))
        assert prune[bins == b].mean() >= 0.1 - 1e-12


def test_depth_bins_follow_eq14():
    sc = small_shell(n=4000, seed=2, deg=0)
    cams = synth.make_cameras_ring(np.random.default_rng(0), 4)
    delta = quantile.depth_proxy(sc, cams)
    bins, p5, p95 = quantile.depth_bins(delta, 16)
    assert p5 == np.quantile(delta, 0.05, method="inverted_cdf")
    assert p95 == np.quantile(delta, 0.95, method="inverted_cdf")
    assert np.all(bins[delta <= p5] == 0) and np.all(bins[delta >= p95] == 15)
    order = np.argsort(delta, kind="stable")
    assert np.all(np.diff(bins[order]) >= 0)                           # monotone in depth
    # about 5% of voxels at each clipped end
    assert 0.04 < (bins == 0).mean() and 0.04 < (bins == 15).mean()


# ------------------------------------------------------- T12 gamma ramp
def test_gamma_schedule_eq9():
    T = 20000
    assert loss.gamma_schedule(0, T) == 0.0
    assert loss.gamma_schedule(0.3 * T - 1, T) == 0.0
    assert loss.gamma_schedule(0.3 * T, T) == 0.0
    assert abs(loss.gamma_schedule(0.45 * T, T) - 0.3) < 1e-12
    assert loss.gamma_schedule(0.6 * T, T) == 0.6
    assert loss.gamma_schedule(T, T) == 0.6
    # continuous at both knots
    for t in (0.3 * T, 0.6 * T):
        assert abs(loss.gamma_schedule(t - 1e-6, T) - loss.gamma_schedule(t, T)) < 1e-6


# ------------------------------------------- depth proxy by hand (R16)
def _camera_facing(centre, forward, dist, fx, fy, width=64, height=48, roll=0.0):
    """A pinhole camera whose optical axis passes through `centre` at depth
    `dist` along the unit `forward` direction; rows of R are right, down,
    forward (turned by `roll` about the axis), so R is not axis-aligned."""
    f = np.asarray(forward, np.float64)
    f /= np.linalg.norm(f)
    r = np.cross(f, [0.0, 1.0, 0.0])
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    cr, sr = math.cos(roll), math.sin(roll)
    r, d = cr * r + sr * d, -sr * r + cr * d
    o = np.asarray(centre, np.float64) - dist * f
    return Camera(R=np.stack([r, d, f]).astype(np.float32), o=o.astype(np.float32),
                  fx=float(np.float32(fx)), fy=float(np.float32(fy)), cx=width / 2.0,
                  cy=height / 2.0, width=width, height=height)


def test_depth_proxy_hand_values():
    # two level-3 leaves of the root [-1, 1]^3 (edge 1/4): centres are exact
    ijk = np.array([[3, 5], [2, 6], [4, 1]], np.uint16)
    sc = Scene(root_min=np.array([-1, -1, -1], np.float32), root_size=2.0, ijk=ijk,
               level=np.array([3, 3], np.uint8), density=np.ones((8, 2), np.float32),
               sh=np.ones((3, 2), np.float32), sh_degree=0)
    centre = np.array([-1 + 0.25 * (3 + 0.5), -1 + 0.25 * (2 + 0.5), -1 + 0.25 * (4 + 0.5)])
    fwd_a = np.array([0.3, -0.2, 0.9])
    fwd_b = np.array([-0.7, 0.4, 0.2])
    # A: on axis at depth 3.0, fx != fy; B: on axis at depth 2.0 with a larger fx
    # (smaller spacing 2/900 < 3/700); C: the voxel lies behind it (z < 0)
    cam_a = _camera_facing(centre, fwd_a, 3.0, fx=700.0, fy=350.0, roll=0.4)
    cam_b = _camera_facing(centre, fwd_b, 2.0, fx=900.0, fy=1500.0, roll=-1.1)
    cam_c = _camera_facing(centre, -fwd_a, -2.5, fx=50.0, fy=50.0)
    delta = quantile.depth_proxy(sc, [cam_a])
    assert abs(delta[0] - 3.0 / 700.0) < 3e-6 * (3.0 / 700.0)        # depth / fx, not fy
    # the spacing uses the camera-space depth, not the distance: the second
    # voxel is off the axis, and its depth is the projection on the axis
    c2 = np.array([-1 + 0.25 * 5.5, -1 + 0.25 * 6.5, -1 + 0.25 * 1.5])
    f = fwd_a / np.linalg.norm(fwd_a)
    z2 = float(f @ (c2 - (centre - 3.0 * f)))
    assert abs(delta[1] - z2 / 700.0) < 3e-6 * abs(z2 / 700.0)
    assert abs(np.linalg.norm(c2 - (centre - 3.0 * f)) - z2) > 0.05
    both = quantile.depth_proxy(sc, [cam_a, cam_b])
    assert abs(both[0] - 2.0 / 900.0) < 3e-6 * (2.0 / 900.0)         # minimum over views
    swapped = quantile.depth_proxy(sc, [cam_b, cam_a])
    assert swapped[0] == both[0]
    behind = quantile.depth_proxy(sc, [cam_c])
    assert np.all(np.isinf(behind))                                   # no view in front
    assert quantile.depth_proxy(sc, [cam_c, cam_a])[0] == delta[0]


# ------------------------------------------ tile numbering by hand (R6)
def test_tile_lists_global_numbering_by_hand():
    # view 0 is 40 x 20 px (3 x 2 tiles of 16), view 1 is 20 x 40 px (2 x 3):
    # global tile id = base(view) + ty * tiles_x(view) + tx, bases 0 and 6
    cams = [Camera(R=np.eye(3, dtype=np.float32), o=np.zeros(3, np.float32), fx=1.0, fy=1.0,
                   cx=0.0, cy=0.0, width=40, height=20),
            Camera(R=np.eye(3, dtype=np.float32), o=np.zeros(3, np.float32), fx=1.0, fy=1.0,
                   cx=0.0, cy=0.0, width=20, height=40)]
    n = 4
    vis = np.zeros((2, n), np.uint8)
    rect = np.zeros((2, n, 4), np.int32)
    code = np.zeros((2, n), np.uint64)
    # (view, voxel): pixel-centre rect (x0, x1, y0, y1), code
    recs = {(0, 0): ((17, 33, 0, 5), 50), (0, 1): ((20, 22, 2, 3), 7),
            (0, 2): ((0, 39, 19, 19), 3), (1, 1): ((0, 3, 16, 35), 9),
            (1, 3): ((19, 19, 39, 39), 1)}
    for (v, i), (r, c) in recs.items():
        vis[v, i] = 1
        rect[v, i] = r
        code[v, i] = c
    start, ids, keys = oracle.tile_lists(cams, vis, rect, code, 16)
    expect = {1: [1, 0], 2: [0], 3: [2], 4: [2], 5: [2], 8: [1], 10: [1], 11: [3]}
    assert start.shape[0] == 13
    for t in range(12):
        got = list(ids[start[t]:start[t + 1]])
        assert got == expect.get(t, []), (t, got)
        tile_of_key = keys[start[t]:start[t + 1]] >> np.uint64(36)
        assert np.all(tile_of_key == t)


# --------------------------------------------- colour clamp by hand (R8)
def test_negative_colour_channel_is_clamped():
    sigma = float(np.float32(0.9))
    col = (float(np.float32(-0.3)), float(np.float32(0.5)), float(np.float32(0.0)))
    bg = (0.25, 0.5, 0.75)
    sc = one_voxel_scene(sigma, col)
    cam = axis_camera((0.0, 0.0, -3.0), (0.0, 0.0, 0.0))
    out = oracle.render(sc, [cam], bg=bg)
    A = out["alpha"]
    rgb = out["views"][0].reshape(3, -1)
    assert A.max() > 0.3
    # the clamped channel shows only the background through T_K
    assert np.max(np.abs(rgb[0] - (1.0 - A) * bg[0])) < 1e-14
    assert np.max(np.abs(rgb[1] - (A * col[1] + (1.0 - A) * bg[1]))) < 1e-14
    assert np.max(np.abs(rgb[2] - (1.0 - A) * bg[2])) < 1e-14
    # no gradient reaches a coefficient through a clamped (or zero) channel;
    # the open channel's constant term gets sum_p g_p w_p with w_p = A_p
    rng = np.random.default_rng(3)
    g = rng.normal(0.0, 1.0, 3 * A.shape[0])
    _, dsh = oracle.backward(sc, [cam], g, bg=bg)
    assert dsh[0, 0] == 0.0 and dsh[2, 0] == 0.0
    gv = g.reshape(3, -1)
    assert abs(dsh[1, 0] - float(gv[1] @ A)) < 1e-10 * max(1.0, abs(dsh[1, 0]))
