"""Parity of the auxiliary channels and terms (eq. 6 and 17 name them;
readings in include/litevoxel.h and oracle/) at the benchmark's full size
(1M voxels, SH3, 8 ring views, 9.37 MP) in the autotuned launch
configuration, over every pixel, one step at a time on shared inputs:
  - the distortion, normal and median-depth channels of the GPU forward
    against the oracle's render;
  - the four image terms and their image gradients, both sides on the
    oracle's channels (rounded to binary32);
  - one backward with every channel's gradient, both sides driven by the
    oracle's upstream gradients of the objective the benchmark's auxiliary
    step differentiates (inverse-Sobel weighted L1 plus the three terms).
The depth-normal term's depth gradient carries 1 / |e_y x e_x| of each
stencil, so near-degenerate stencils amplify a 1e-5 difference between two
depth maps into a large one: the end-to-end chain (each side on its own
images) is compared at a smaller size (test_gpu_aux), here each step takes
the same inputs on both sides."""
import numpy as np
import pytest

import oracle
from oracle import aux as oaux
from oracle import loss as oloss
import synth
from gpu_helpers import GRAD_TOL, IMG_TOL, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu

GAMMA, FORM, EPS = 0.4, 0, 1e-3
LAM = (0.01, 0.05, 1.0)   # transmittance concentration, depth-normal, distortion
LAM_NM = 0.05             # median depth-normal


@pytest.fixture(scope="module")
def ring_aux():
    import paper_2511_02510_amd as lv
    import torch
    ctx = lv.Context(0)
    say("full size, auxiliary channels: generating the 1M-voxel ring workload")
    scene, cams, targets = synth.make_config("ring1m")
    dev = ctx.device
    vox = lv.Voxels.from_scene(scene, dev)
    frame = lv.Frame(cams, dev)
    best, _ = lv.autotune(ctx, vox, frame, reps=2)
    say(f"  autotuned tile={best.tile} chunk={best.chunk} chunk_bwd={best.chunk_bwd}")
    P = frame.P
    r = lv.Renderer(ctx, vox, frame, lv.settings(tile=best.tile, chunk=best.chunk,
                                                 chunk_bwd=best.chunk_bwd,
                                                 pair_capacity=best.pair_capacity))
    rgb, depth, alpha = r.new_outputs()
    dist, normal = torch.empty(P, device=dev), torch.empty(3 * P, device=dev)
    mdepth = torch.empty(P, device=dev)
    wmax = torch.zeros(vox.n, device=dev)
    say("  forward with the auxiliary channels")
    r.forward(rgb, depth, alpha, wmax, dist=dist, normal=normal, mdepth=mdepth)
    torch.cuda.synchronize()
    f64 = lambda t: t.cpu().numpy().astype(np.float64)
    out = dict(ctx=ctx, r=r, vox=vox, frame=frame, scene=scene, cams=cams, targets=targets,
               depth_dev=depth, rgb=f64(rgb), depth=f64(depth), alpha=f64(alpha), dist=f64(dist),
               normal=f64(normal), mdepth=f64(mdepth))
    say("  oracle: render with the auxiliary channels, every pixel")
    out["ref"] = oracle.render_aux(scene, cams)
    out["ref"]["mdepth"] = oracle.median_depth(scene, cams)
    yield out
    del out["r"], out["vox"], out["frame"], out["depth_dev"]
    ctx.close()
    torch.cuda.empty_cache()


def test_fullsize_aux_channels_every_pixel(ring_aux):
    ref = ring_aux["ref"]
    errs = {k: float(np.abs(ring_aux[k] - ref[k]).max())
            for k in ("rgb", "depth", "alpha", "dist", "normal")}
    say(f"full size: all {ref['depth'].shape[0]} pixels, max abs " +
        " ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    assert all(v <= IMG_TOL for v in errs.values()), errs
    from test_gpu_aux import check_mdepth
    check_mdepth(ring_aux["mdepth"], ring_aux["scene"], ring_aux["cams"])
    # the workload's corner densities are drawn independently, so voxel
    # normals point every way and the blended normal stays short
    assert ref["dist"].max() > 1e-3 and np.abs(ref["normal"]).max() > 0.05


def test_fullsize_aux_terms_on_shared_channels(ring_aux):
    import torch
    import paper_2511_02510_amd as lv
    ref, cams, frame = ring_aux["ref"], ring_aux["cams"], ring_aux["frame"]
    dev, P, V = ring_aux["ctx"].device, frame.P, frame.n_views
    ch = {k: ref[k].astype(np.float32) for k in ("depth", "alpha", "normal", "dist", "mdepth")}
    La, ga, gd, gn, gl = oaux.aux_losses(ch["depth"], ch["alpha"], ch["normal"], ch["dist"],
                                         cams, *LAM, mdepth=ch["mdepth"], lam_nm=LAM_NM)
    loss = torch.empty(4 * V, device=dev)
    g = [torch.empty(P, device=dev), torch.empty(P, device=dev), torch.empty(3 * P, device=dev),
         torch.empty(P, device=dev)]
    t = {k: to_dev(v, dev) for k, v in ch.items()}
    lv.aux_loss(ring_aux["ctx"], frame, t["depth"], t["alpha"], t["normal"], t["dist"], *LAM,
                loss, *g, mdepth=t["mdepth"], lam_nm=LAM_NM)
    torch.cuda.synchronize()
    Lg = loss.cpu().numpy().astype(np.float64).reshape(V, 4)
    e_L = float(np.max(np.abs(Lg - La) / np.maximum(np.abs(La), 1e-12)))
    errs = {name: rel_l2(x.cpu().numpy().astype(np.float64), r) for name, x, r in
            zip(("d_alpha", "d_depth", "d_normal", "d_dist"), g, (ga, gd, gn, gl))}
    say(f"full size: auxiliary terms of 8 views, max rel {e_L:.2e}; image gradients rel L2: " +
        " ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    assert e_L <= 1e-4 and La[:, 3].min() > 0.0
    assert all(v <= GRAD_TOL for v in errs.values()), errs


def test_fullsize_aux_backward_whole_gradient(ring_aux):
    import torch
    ref, cams = ring_aux["ref"], ring_aux["cams"]
    _, ga, gd, gn, gl = oaux.aux_losses(ref["depth"], ref["alpha"], ref["normal"], ref["dist"],
                                        cams, *LAM, mdepth=ref["mdepth"], lam_nm=LAM_NM)
    g_rgb = []
    for v in range(len(cams)):
        w = oloss.lf_weight(ring_aux["targets"][v], GAMMA, form=FORM, eps=EPS)
        _, gv = oloss.l1_loss_grad(ref["views"][v], ring_aux["targets"][v], w)
        g_rgb.append(gv)
    g_rgb = oracle.join_views(g_rgb)
    dev, vox, r = ring_aux["ctx"].device, ring_aux["vox"], ring_aux["r"]
    dd, dsh = torch.empty_like(vox.density), torch.empty_like(vox.sh)
    up = [to_dev(a, dev) for a in (g_rgb, gd, ga, gl, gn)]
    r.backward_aux(up[0], up[1], up[2], ring_aux["depth_dev"], up[3], up[4], dd, dsh)
    torch.cuda.synchronize()
    say("full size: oracle backward with every channel's gradient, every pixel")
    dd_r, dsh_r = oracle.backward_aux(ring_aux["scene"], cams, g_rgb, gd, ga, gl, gn)
    f64 = lambda t: t.cpu().numpy().astype(np.float64)
    e1, e2 = rel_l2(f64(dd), dd_r), rel_l2(f64(dsh), dsh_r)
    say(f"  whole gradient rel L2: density {e1:.2e} sh {e2:.2e}")
    assert e1 <= GRAD_TOL and e2 <= GRAD_TOL
    assert np.count_nonzero(dd_r) > 1000000
