"""Pins of the oracle's auxiliary channels and terms (eq. 6 and 17 name them;
the readings are in oracle/raster_ref.cpp and oracle/aux.py): closed forms on
one and two voxels, the voxel normal against a numerical derivative of the
trilinear field, a plane's depth normal, and central finite differences of
the analytic gradients.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from oracle import aux
import synth
from synth.scenes import Scene, look_at

from test_oracle_pins import GOLDEN, axis_camera, one_voxel_scene


def test_distortion_single_voxel_is_the_self_term():
    sigma = float(np.float32(1.3))
    sc = one_voxel_scene(sigma, (0.5, 0.5, 0.5))
    cam = axis_camera((0.0, 0.0, -3.0), (0.0, 0.0, 0.0))
    out = oracle.render_aux(sc, [cam])
    a = 1 - math.exp(-sigma)          # central ray: chord of length 1
    k = 32 * 65 + 32
    assert abs(out["dist"][k] - a * a / 3.0) < 1e-14
    # the other channels are the plain renderer's
    ref = oracle.render(sc, [cam])
    for key in ("rgb", "depth", "alpha", "wmax"):
        assert np.array_equal(out[key], ref[key])


def test_distortion_two_voxels_closed_form():
    g = GOLDEN["two_voxel_stack"]
    f = lambda x: float(np.float32(x))
    s1, s2 = f(g["sigma1"]), f(g["sigma2"])
    sc = Scene(root_min=np.array([-1, -1, -1], np.float32), root_size=2.0,
               ijk=np.array([[0, 0], [0, 0], [0, 1]], np.uint16),
               level=np.array([1, 1], np.uint8),
               density=np.array([[s1, s2]] * 8, np.float32),
               sh=np.full((3, 2), 0.5, np.float32), sh_degree=0)
    cam = axis_camera((-0.5, -0.5, -4.0), (-0.5, -0.5, 0.0))
    out = oracle.render_aux(sc, [cam])
    w1 = 1 - math.exp(-s1)
    w2 = (1 - w1) * (1 - math.exp(-s2))
    t1, t2 = g["t_mid1"], g["t_mid2"]     # chords of length 1 each
    want = 2 * w1 * w2 * (t2 - t1) + (w1 * w1 + w2 * w2) / 3.0
    assert abs(out["dist"][32 * 65 + 32] - want) < 1e-12
    # uniform densities: no gradient, no normal
    assert np.all(out["normal"] == 0.0)


def test_normal_of_a_density_ramp_along_x():
    # corner values a + b x_bit: the gradient points along +x, the normal along -x
    dens = np.array([0.5 + 1.5 * (c & 1) for c in range(8)], np.float32)
    sc = one_voxel_scene(dens, (0.2, 0.4, 0.6))
    cam = axis_camera((0.0, 0.0, -3.0), (0.0, 0.0, 0.0))
    out = oracle.render_aux(sc, [cam])
    N = out["normal"].reshape(3, 65, 65)
    A = out["alpha"].reshape(65, 65)
    hit = A > 0
    assert hit.sum() > 100
    assert np.allclose(N[0][hit], -A[hit], atol=1e-14, rtol=0)
    assert np.all(N[1] == 0.0) and np.all(N[2] == 0.0)


def trilinear(dens, u):
    s = 0.0
    for c in range(8):
        w = 1.0
        for a in range(3):
            w *= u[a] if (c >> a) & 1 else 1.0 - u[a]
        s += dens[c] * w
    return s


def test_normal_equals_the_numerical_gradient_at_the_centre():
    rng = np.random.default_rng(3)
    dens = rng.uniform(0.1, 3.0, 8).astype(np.float32)
    sc = one_voxel_scene(dens, (0.5, 0.5, 0.5))
    cam = axis_camera((0.0, 0.0, -3.0), (0.0, 0.0, 0.0))
    out = oracle.render_aux(sc, [cam])
    # central differences of the trilinear field at the centre (exact: the
    # field is linear along each axis)
    d64 = dens.astype(np.float64)
    g = np.array([(trilinear(d64, [0.5 + (a == 0) * 0.25, 0.5 + (a == 1) * 0.25, 0.5 + (a == 2) * 0.25])
                   - trilinear(d64, [0.5 - (a == 0) * 0.25, 0.5 - (a == 1) * 0.25, 0.5 - (a == 2) * 0.25]))
                  / 0.5 for a in range(3)])
    n = -g / np.linalg.norm(g)
    k = 32 * 65 + 32
    a = out["alpha"][k]
    got = out["normal"].reshape(3, -1)[:, k]
    assert np.allclose(got, a * n, atol=1e-13, rtol=0)


def _aux_loss(sc, cams, gr, gd, ga, gl, gn):
    out = oracle.render_aux(sc, cams)
    return (float(gr @ out["rgb"]) + float(gd @ out["depth"]) + float(ga @ out["alpha"])
            + float(gl @ out["dist"]) + float(gn @ out["normal"])), out


def test_aux_gradient_matches_central_differences():
    rng = np.random.default_rng(17)
    sc = synth.make_scene_shell(np.random.default_rng(5), 1500, 4, 6, sh_degree=2, clutter_frac=0.0)
    cams = [look_at((1.2, 0.9, 2.0), 40, 30), look_at((-2.0, 0.5, 1.0), 36, 28)]
    P = sum(c.npix for c in cams)
    gr, gn = rng.normal(0, 1e-2, 3 * P), rng.normal(0, 1e-2, 3 * P)
    gd, ga, gl = rng.normal(0, 1e-3, P), rng.normal(0, 1e-2, P), rng.normal(0, 1e-1, P)
    L0, out = _aux_loss(sc, cams, gr, gd, ga, gl, gn)
    dd, dsh = oracle.backward_aux(sc, cams, gr, gd, ga, gl, gn)
    raw0, _ = oracle.voxel_colours(sc, cams)
    hit = np.nonzero(out["wmax"] > 1e-3)[0]
    h = 1e-3
    fd, an = [], []
    tries = 0
    while len(fd) < 64 and tries < 400:
        tries += 1
        v = int(rng.choice(hit))
        arr, row = ("density", int(rng.integers(0, 8))) if len(fd) < 40 else ("sh", int(rng.integers(0, 27)))
        vals, ok = [], True
        for sgn in (+1, -1):
            s2 = synth.scene_subset(sc, np.arange(sc.n))
            getattr(s2, arr)[row, v] += np.float32(sgn * h)
            vals.append(_aux_loss(s2, cams, gr, gd, ga, gl, gn)[0])
            raw2, _ = oracle.voxel_colours(s2, cams)
            if np.any((raw2[:, v] > 0) != (raw0[:, v] > 0)):
                ok = False
        if not ok:
            continue
        x = getattr(sc, arr)[row, v]
        hp = float(np.float32(x + np.float32(h)) - x)
        hm = float(x - np.float32(x - np.float32(h)))
        fd.append((vals[0] - vals[1]) / (hp + hm))
        an.append(dd[row, v] if arr == "density" else dsh[row, v])
    assert len(fd) == 64
    fd, an = np.array(fd), np.array(an)
    rel = np.linalg.norm(fd - an) / np.linalg.norm(an)
    assert rel < 1e-4, rel
    # with no auxiliary upstream the gradient is the plain backward's
    dd0, dsh0 = oracle.backward_aux(sc, cams, gr, gd, ga)
    ddr, dshr = oracle.backward(sc, cams, gr, gd, ga)
    assert np.allclose(dd0, ddr, rtol=1e-12, atol=1e-18) and np.allclose(dsh0, dshr, rtol=1e-12, atol=1e-18)


def _plane_depth(cam, p0, nrm):
    d = aux.pixel_dirs(cam)
    nrm = np.asarray(nrm, np.float64) / np.linalg.norm(nrm)
    t = ((np.asarray(p0) - np.asarray(cam.o)) @ nrm) / (d @ nrm)
    return t, nrm


def test_depth_normal_of_a_plane_faces_the_camera():
    cam = look_at((0.3, 0.4, -2.5), 33, 29)
    t, nrm = _plane_depth(cam, (0.0, 0.0, 0.0), (0.2, -0.3, -1.0))
    m, _, _, _ = aux.depth_normals(t, cam)
    assert np.allclose(m, nrm, atol=1e-9, rtol=0)
    # the same plane seen from the other side: the normal flips towards that camera
    cam2 = look_at((-0.3, -0.2, 2.5), 33, 29)
    t2, _ = _plane_depth(cam2, (0.0, 0.0, 0.0), (0.2, -0.3, -1.0))
    m2, _, _, _ = aux.depth_normals(t2, cam2)
    assert np.allclose(m2, -nrm, atol=1e-9, rtol=0)


def test_aux_losses_closed_forms_and_sign():
    cams = [look_at((0.3, 0.4, -2.5), 9, 7), look_at((2.0, 0.1, 0.5), 6, 5)]
    P = sum(c.npix for c in cams)
    rng = np.random.default_rng(9)
    A = rng.uniform(0, 1, P)
    dist = rng.uniform(0, 0.1, P)
    D = np.concatenate([_plane_depth(c, (0, 0, 0), (0.2, -0.3, -1.0))[0].ravel() for c in cams])
    # normals of length at most A: the depth-normal term is non-negative
    raw = rng.normal(0, 1, (3, P))
    Nn = A * rng.uniform(0, 1, P) * raw / np.linalg.norm(raw, axis=0)
    N = np.concatenate([Nn[:, int(o0):int(o1)].ravel() for o0, o1 in
                        zip(oracle.pix_offsets(cams)[:-1], oracle.pix_offsets(cams)[1:])])
    L, g_a, g_d, g_n, g_l = aux.aux_losses(D, A, N, dist, cams, 0.7, 1.3, 2.0)
    off = oracle.pix_offsets(cams)
    for v, c in enumerate(cams):
        sl = slice(int(off[v]), int(off[v + 1]))
        assert abs(L[v, 0] - 0.7 * np.mean(A[sl] * (1 - A[sl]))) < 1e-15
        assert abs(L[v, 2] - 2.0 * np.mean(dist[sl])) < 1e-15
        assert L[v, 1] >= 0.0
        assert np.allclose(g_l[sl], 2.0 / c.npix)
    # transmittance concentration: zero at A in {0, 1}, largest at 1/2
    L01, ga01, _, _, _ = aux.aux_losses(D, np.round(A), N * 0, dist * 0, cams, 1.0, 0.0, 0.0)
    assert np.all(L01[:, 0] == 0.0)
    assert np.allclose(ga01, np.where(np.round(A) == 0, 1.0, -1.0) /
                       np.concatenate([[c.npix] * c.npix for c in cams]))


def test_aux_losses_gradients_by_finite_differences():
    cams = [look_at((0.3, 0.4, -2.5), 9, 7), look_at((2.0, 0.1, 0.5), 6, 5)]
    P = sum(c.npix for c in cams)
    rng = np.random.default_rng(11)
    D = np.concatenate([_plane_depth(c, (0, 0, 0), (0.2, -0.3, -1.0))[0].ravel() for c in cams])
    D = D + rng.normal(0, 0.05, P)                 # a rough surface
    A = rng.uniform(0.2, 0.9, P)
    N = rng.normal(0, 0.3, 3 * P)
    dist = rng.uniform(0, 0.1, P)
    lam = (0.7, 1.3, 2.0)
    _, g_a, g_d, g_n, g_l = aux.aux_losses(D, A, N, dist, cams, *lam)
    tot = lambda D_, A_, N_, l_: float(np.sum(aux.aux_losses(D_, A_, N_, l_, cams, *lam)[0]))
    h = 1e-6
    for arr, g, idx in (("D", g_d, rng.integers(0, P, 25)), ("A", g_a, rng.integers(0, P, 10)),
                        ("N", g_n, rng.integers(0, 3 * P, 25)), ("l", g_l, rng.integers(0, P, 5))):
        for i in idx:
            xs = {"D": D.copy(), "A": A.copy(), "N": N.copy(), "l": dist.copy()}
            xs[arr][i] += h
            lp = tot(xs["D"], xs["A"], xs["N"], xs["l"])
            xs[arr][i] -= 2 * h
            lm = tot(xs["D"], xs["A"], xs["N"], xs["l"])
            assert abs((lp - lm) / (2 * h) - g[i]) < 1e-7 * max(1.0, abs(g[i])), (arr, i)


# ------------------------------------------------------------ median depth
def test_median_depth_single_voxel_either_side_of_one_half():
    # constant density sigma over a chord of length 1: T = exp(-sigma); half
    # the opacity is reached exactly when sigma >= ln 2
    cam = axis_camera((0.0, 0.0, -3.0), (0.0, 0.0, 0.0))
    k = 32 * 65 + 32
    for sigma, want in ((math.log(2.0) + 0.01, 3.0), (math.log(2.0) - 0.01, 0.0)):
        s = float(np.float32(sigma))
        sc = one_voxel_scene(s, (0.5, 0.5, 0.5))
        md = oracle.median_depth(sc, [cam])
        assert abs(md[k] - want) < 1e-12, (sigma, md[k])
    # a pixel that misses the voxel has no median depth
    assert md[0] == 0.0


def test_median_depth_two_voxels_picks_the_crossing_hit():
    g = GOLDEN["two_voxel_stack"]
    cam = axis_camera((-0.5, -0.5, -4.0), (-0.5, -0.5, 0.0))
    k = 32 * 65 + 32
    # exp(-0.4) > 1/2 > exp(-0.9): the second hit takes T below one half;
    # exp(-0.8) < 1/2: the first one does
    for s1, s2, want in ((0.4, 0.5, g["t_mid2"]), (0.8, 0.5, g["t_mid1"]), (0.2, 0.3, 0.0)):
        sc = Scene(root_min=np.array([-1, -1, -1], np.float32), root_size=2.0,
                   ijk=np.array([[0, 0], [0, 0], [0, 1]], np.uint16),
                   level=np.array([1, 1], np.uint8),
                   density=np.array([[s1, s2]] * 8, np.float32),
                   sh=np.full((3, 2), 0.5, np.float32), sh_degree=0)
        assert abs(oracle.median_depth(sc, [cam])[k] - want) < 1e-12, (s1, s2)


def test_median_depth_normal_term_is_the_mean_term_on_the_same_map():
    """With the median-depth map equal to the depth map, the median term is
    the mean term (its weight swapped) with the same alpha and normal
    gradients; it passes no depth gradient."""
    cams = [look_at((0.3, 0.4, -2.5), 9, 7), look_at((2.0, 0.1, 0.5), 6, 5)]
    P = sum(c.npix for c in cams)
    rng = np.random.default_rng(12)
    D = np.concatenate([_plane_depth(c, (0, 0, 0), (0.2, -0.3, -1.0))[0].ravel() for c in cams])
    D = D + rng.normal(0, 0.05, P)
    A = rng.uniform(0.2, 0.9, P)
    N = rng.normal(0, 0.3, 3 * P)
    dist = np.zeros(P)
    Ln, ga_n, gd_n, gn_n, _ = aux.aux_losses(D, A, N, dist, cams, 0.0, 0.8, 0.0)
    Lm, ga_m, gd_m, gn_m, _ = aux.aux_losses(D, A, N, dist, cams, 0.0, 0.0, 0.0, mdepth=D,
                                             lam_nm=0.8)
    assert np.allclose(Lm[:, 3], Ln[:, 1], rtol=1e-14, atol=0.0)
    assert np.all(Lm[:, :3] == 0.0)
    assert np.allclose(ga_m, ga_n, rtol=1e-14, atol=0.0)
    assert np.allclose(gn_m, gn_n, rtol=1e-14, atol=0.0)
    assert np.all(gd_m == 0.0) and np.any(gd_n != 0.0)
    # finite differences in alpha and normal of the median term alone
    M = D + rng.normal(0, 0.02, P)
    _, ga, _, gn, _ = aux.aux_losses(D, A, N, dist, cams, 0.0, 0.0, 0.0, mdepth=M, lam_nm=1.7)
    tot = lambda A_, N_: float(np.sum(aux.aux_losses(D, A_, N_, dist, cams, 0.0, 0.0, 0.0,
                                                     mdepth=M, lam_nm=1.7)[0]))
    h = 1e-6
    for i in rng.integers(0, P, 10):
        Ap, Am = A.copy(), A.copy()
        Ap[i] += h
        Am[i] -= h
        assert abs((tot(Ap, N) - tot(Am, N)) / (2 * h) - ga[i]) < 1e-7
    for i in rng.integers(0, 3 * P, 20):
        Np, Nm = N.copy(), N.copy()
        Np[i] += h
        Nm[i] -= h
        assert abs((tot(A, Np) - tot(A, Nm)) / (2 * h) - gn[i]) < 1e-7
