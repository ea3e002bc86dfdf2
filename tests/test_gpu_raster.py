"""GPU parity of the rasterizer (through the C-ABI) against the FP64 oracle:
keys and per-tile order bit-exact, images <= 1e-4 max abs, w_max <= 1e-5,
gradients <= 1e-3 relative L2, on seeded synthetic scenes."""
import numpy as np
import pytest

import oracle
import synth
from synth.scenes import Scene, look_at
from gpu_helpers import (GRAD_TOL, WMAX_TOL, check_images, check_keys, random_grads, rel_l2,
                         run_gpu, say, small_shell)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_02510_amd as lv
    c = lv.Context(0)
    yield c
    c.close()


# ------------------------------------------------------------------ keys
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_keys_grid4k(ctx, tile):
    scene, cams, _ = synth.make_config("grid4k")
    say(f"keys grid4k tile={tile}")
    g = run_gpu(ctx, scene, cams, tile=tile)
    q = check_keys(g["bins"], scene, cams, tile)
    assert q > 4096


def test_keys_shell_two_uneven_views(ctx):
    scene = small_shell(20000, seed=1, lmin=5, lmax=9, clutter=0.1)
    cams = [look_at((1.9, 0.7, 1.2), 97, 61), look_at((-0.4, 1.1, -2.3), 128, 80)]
    say("keys shell 20k, 2 views 97x61 + 128x80")
    g = run_gpu(ctx, scene, cams, tile=16)
    check_keys(g["bins"], scene, cams, 16)


def test_keys_camera_inside_root_cube(ctx):
    # voxels straddling the camera plane cover the whole image
    scene = small_shell(5000, seed=2, lmin=4, lmax=7, clutter=0.5)
    cams = [look_at((0.05, 0.02, 0.79), 50, 40, target=(0.3, 0.1, -0.5))]
    say("keys camera inside the root cube")
    g = run_gpu(ctx, scene, cams, tile=8)
    check_keys(g["bins"], scene, cams, 8)
    vis, rect, _ = oracle.project_keys(scene, cams)
    full = (rect[0, :, 0] == 0) & (rect[0, :, 1] == 49) & (rect[0, :, 2] == 0) & (rect[0, :, 3] == 39)
    assert np.any(full & (vis[0] == 1))


def test_keys_eye_on_split_planes(ctx):
    # the visibility code behind the front-to-back order of eq. 2-4 compares
    # the eye with the split plane of every level: eyes exactly on planes of
    # levels 1, 3, 9 and 12, one ulp above and below them, and outside the
    # root cube on either side, with a root cube whose size is not a power of
    # two and leaves down to level 12
    scene = small_shell(20000, seed=6, lmin=5, lmax=12, clutter=0.3)
    scene.root_min = np.array([-1.3, -1.05, -1.7], np.float32)
    scene.root_size = 2.7
    f32 = np.float32

    def plane(a, k):
        return f32(scene.root_min[a] + f32(np.ldexp(f32(f32(k) * f32(scene.root_size)), -12)))

    on = np.array([plane(0, 2048), plane(1, 1536), plane(2, 1237)], np.float32)
    up = np.nextafter(on, np.float32(np.inf))
    down = np.nextafter(on, np.float32(-np.inf))
    outside = np.array([scene.root_min[0] - 0.5, scene.root_min[1] + 2.7 + 0.3, plane(2, 3000)],
                       np.float32)
    centre = scene.root_min.astype(np.float64) + 1.35
    cams = [look_at(o.astype(np.float64), 320, 240, target=tuple(centre + [0.31, -0.17, 0.23]))
            for o in (on, up, down, outside)]
    say("keys with the eye on split planes, 4 views, leaves to level 12")
    g = run_gpu(ctx, scene, cams, tile=16)
    check_keys(g["bins"], scene, cams, 16)
    assert int(scene.level.max()) == 12


def test_keys_long_tile_lists_use_merge_path(ctx):
    # 32^3 uniform grid seen small: single tiles hold more than 4096 voxels
    rng = np.random.default_rng(3)
    scene = synth.make_scene_grid(rng, res_level=5, sh_degree=0)
    cams = [look_at((2.0, 1.4, 2.9), 64, 64)]
    say("keys 32^3 grid, long lists")
    g = run_gpu(ctx, scene, cams, tile=32)
    ts = g["bins"]["tile_start"]
    assert np.diff(ts).max() > 4096
    check_keys(g["bins"], scene, cams, 32)


# -------------------------------------------------------------- forward
@pytest.mark.parametrize("tile,chunk", [(16, 64), (8, 128), (32, 256)])
def test_forward_grid4k(ctx, tile, chunk):
    scene, cams, _ = synth.make_config("grid4k")
    say(f"forward grid4k tile={tile} chunk={chunk}")
    g = run_gpu(ctx, scene, cams, tile=tile, chunk=chunk, export=False)
    ref = oracle.render(scene, cams)
    check_images(g, ref)
    assert np.abs(g["wmax"] - ref["wmax"]).max() <= WMAX_TOL


def test_forward_shell_sh3_background(ctx):
    scene = small_shell(30000, seed=4, lmin=5, lmax=9)
    cams = [look_at((2.2, 0.4, 1.1), 83, 67), look_at((0.3, -2.0, 1.5), 40, 96)]
    bg = (0.2, 0.5, 0.9)
    say("forward shell 30k SH3, 2 ragged views, background")
    g = run_gpu(ctx, scene, cams, tile=16, chunk=128, bg=bg, export=False)
    ref = oracle.render(scene, cams, bg=bg)
    check_images(g, ref)
    assert np.abs(g["wmax"] - ref["wmax"]).max() <= WMAX_TOL


def test_forward_wmax_accumulates_across_calls(ctx):
    scene, cams, _ = synth.make_config("grid4k")
    prior = np.random.default_rng(5).uniform(0, 0.5, scene.n)
    say("forward w_max max-combined with the caller's buffer")
    g = run_gpu(ctx, scene, cams, export=False, wmax_in=prior)
    ref = oracle.render(scene, cams, wmax_in=prior)
    assert np.abs(g["wmax"] - ref["wmax"]).max() <= WMAX_TOL


def test_forward_empty_scene_and_tiny_views(ctx):
    empty = Scene(root_min=np.array([-1, -1, -1], np.float32), root_size=2.0,
                  ijk=np.zeros((3, 0), np.uint16), level=np.zeros(0, np.uint8),
                  density=np.zeros((8, 0), np.float32), sh=np.zeros((3, 0), np.float32), sh_degree=0)
    cams = [look_at((2.0, 1.0, 1.5), 1, 1), look_at((2.0, 1.0, 1.5), 19, 7)]
    say("forward empty scene, 1x1 and 19x7 views")
    g = run_gpu(ctx, empty, cams, bg=(0.25, 0.5, 0.75))
    assert np.allclose(g["alpha"], 0.0) and np.allclose(g["depth"], 0.0)
    assert np.allclose(g["rgb"][:3], [0.25, 0.5, 0.75])
    scene = small_shell(3000, seed=6, lmin=4, lmax=6)
    g = run_gpu(ctx, scene, cams, tile=32, export=False)
    ref = oracle.render(scene, cams)
    check_images(g, ref)


def test_forward_camera_inside_scene(ctx):
    scene = small_shell(5000, seed=2, lmin=4, lmax=7, clutter=0.5)
    cams = [look_at((0.05, 0.02, 0.79), 50, 40, target=(0.3, 0.1, -0.5))]
    say("forward camera inside the root cube")
    g = run_gpu(ctx, scene, cams, tile=8, export=False)
    ref = oracle.render(scene, cams)
    check_images(g, ref)
    assert np.abs(g["wmax"] - ref["wmax"]).max() <= WMAX_TOL


def test_capacity_overflow_is_reported_and_replanned(ctx):
    import paper_2511_02510_amd as lv
    import torch
    scene, cams, _ = synth.make_config("grid4k")
    say("capacity overflow")
    vox = lv.Voxels.from_scene(scene, ctx.device)
    frame = lv.Frame(cams, ctx.device)
    st = lv.settings(pair_capacity=100)
    ws_bytes, sv_bytes = lv.query_sizes(ctx, vox, frame, st)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=ctx.device)
    sv = torch.empty(sv_bytes, dtype=torch.uint8, device=ctx.device)
    rgb = torch.empty(3 * frame.P, device=ctx.device)
    d = torch.empty(frame.P, device=ctx.device)
    a = torch.empty(frame.P, device=ctx.device)
    w = torch.zeros(vox.n, device=ctx.device)
    lv.forward(ctx, vox, frame, st, ws, sv, rgb, d, a, w)
    fits, need = lv.check_overflow(ctx, vox, frame, st, sv)
    assert not fits and need > 4096
    # the renderer re-plans and the result is exact
    g = run_gpu(ctx, scene, cams, cap=100, export=False)
    assert g["renderer"].st.pair_capacity >= need
    ref = oracle.render(scene, cams)
    check_images(g, ref)
    assert np.abs(g["wmax"] - ref["wmax"]).max() <= WMAX_TOL


# ------------------------------------------------------------- backward
@pytest.mark.parametrize("tile,chunk,chunk_bwd", [(16, 64, 0), (8, 256, 0), (32, 128, 0),
                                                  (16, 128, 64), (16, 64, 256)])
def test_backward_grid4k(ctx, tile, chunk, chunk_bwd):
    # chunk_bwd != chunk: the backward stages its lists with another chunk
    # than the forward that left the per-pixel state
    scene, cams, _ = synth.make_config("grid4k")
    P = cams[0].npix
    grads = random_grads(np.random.default_rng(7), P)
    say(f"backward grid4k tile={tile} chunk={chunk} chunk_bwd={chunk_bwd}")
    g = run_gpu(ctx, scene, cams, tile=tile, chunk=chunk, grads=grads, export=False,
                chunk_bwd=chunk_bwd)
    dd, dsh = oracle.backward(scene, cams, *grads)
    e1, e2 = rel_l2(g["dd"], dd), rel_l2(g["dsh"], dsh)
    say(f"  rel L2: density {e1:.2e} sh {e2:.2e}")
    assert e1 <= GRAD_TOL and e2 <= GRAD_TOL


def test_backward_shell_sh3_two_views(ctx):
    scene = small_shell(30000, seed=8, lmin=5, lmax=9)
    cams = [look_at((2.2, 0.4, 1.1), 83, 67), look_at((0.3, -2.0, 1.5), 40, 96)]
    P = sum(c.npix for c in cams)
    grads = random_grads(np.random.default_rng(9), P)
    bg = (0.1, 0.3, 0.2)
    say("backward shell 30k SH3, 2 ragged views, background")
    g = run_gpu(ctx, scene, cams, tile=16, chunk=64, bg=bg, grads=grads, export=False)
    dd, dsh = oracle.backward(scene, cams, *grads, bg=bg)
    e1, e2 = rel_l2(g["dd"], dd), rel_l2(g["dsh"], dsh)
    say(f"  rel L2: density {e1:.2e} sh {e2:.2e}")
    assert e1 <= GRAD_TOL and e2 <= GRAD_TOL


def test_backward_rgb_only_and_deterministic_forward(ctx):
    scene, cams, _ = synth.make_config("grid4k")
    P = cams[0].npix
    rng = np.random.default_rng(10)
    grads = (rng.normal(0, 1e-3, 3 * P), None, None)
    say("backward rgb-only; forward bit-identical across runs")
    g1 = run_gpu(ctx, scene, cams, grads=grads, export=False)
    g2 = run_gpu(ctx, scene, cams, grads=grads, export=False)
    assert np.array_equal(g1["rgb"], g2["rgb"]) and np.array_equal(g1["wmax"], g2["wmax"])
    assert rel_l2(g1["dd"], g2["dd"]) < 1e-6
    dd, dsh = oracle.backward(scene, cams, grads[0])
    assert rel_l2(g1["dd"], dd) <= GRAD_TOL and rel_l2(g1["dsh"], dsh) <= GRAD_TOL


def test_many_uneven_views_forward_backward_and_keys(ctx):
    # 40 views of odd sizes around the scene in one call: view lookup of every
    # tile, per-view tile and pixel offsets, and the interleaved tile queues
    # over many more tiles than queues
    scene = small_shell(6000, seed=41, lmin=4, lmax=7, clutter=0.2)
    rng = np.random.default_rng(42)
    cams = []
    for i in range(40):
        # generic directions: no camera on a coordinate plane, so no pixel ray
        # runs inside a voxel face (a measure-zero case the FP32 path and the
        # FP64 oracle may resolve to different sides)
        az, el = 2 * np.pi * i / 40 + 0.137, 0.6 * np.sin(1.7 * i) + 0.071
        o = 2.4 * np.array([np.cos(el) * np.cos(az), np.sin(el), np.cos(el) * np.sin(az)])
        cams.append(look_at(tuple(o), int(rng.integers(5, 41)), int(rng.integers(3, 37))))
    say("forward + backward, 40 uneven views")
    P = sum(c.npix for c in cams)
    grads = random_grads(np.random.default_rng(43), P)
    for tile in (8, 16):
        g = run_gpu(ctx, scene, cams, tile=tile, chunk=64, grads=grads)
        check_keys(g["bins"], scene, cams, tile)
        ref = oracle.render(scene, cams)
        check_images(g, ref)
        assert np.abs(g["wmax"] - ref["wmax"]).max() <= WMAX_TOL
        dd, dsh = oracle.backward(scene, cams, *grads)
        assert rel_l2(g["dd"], dd) <= GRAD_TOL and rel_l2(g["dsh"], dsh) <= GRAD_TOL
