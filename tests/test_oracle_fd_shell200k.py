"""Central finite differences of the oracle's analytic gradient on the
200,000-leaf SH-3 shell seen by one 800 x 600 camera, with the ramped
inverse-Sobel weight form (w = (1 + g/g99)^-gamma, eq. 8 normalisation) and the
weighted L1 loss of eq. 10: h = 1e-3 on 64 seeded parameters (32 corner
densities of hit voxels, 32 SH coefficients of visible voxels over all
degrees), rejecting draws whose +-h stencil crosses a kink of the loss (an L1
residual or a clamped colour changing sign).  Only the pixels whose rays can
meet the perturbed voxel change, so each evaluation renders those pixels.
CPU only."""
import numpy as np

import oracle
from oracle import loss
import synth


def _pixel_loss(sc, cam, target_flat, weight_flat, pix):
    """Sum over the listed pixels of w~ mean_ch |C - I| / |P| (their share of eq. 10)."""
    out = oracle.render(sc, [cam], pix_list=pix)
    P = cam.width * cam.height
    rgb = out["rgb"].reshape(3, P)[:, pix]
    res = rgb - target_flat[:, pix]
    return float((weight_flat[pix] * np.abs(res).mean(axis=0)).sum() / P), np.sign(res)


def test_fd_gradient_on_the_200k_shell():
    scene, cams, targets = synth.make_config("shell200k_train")
    cam, target = cams[0], targets[0]
    P = cam.width * cam.height
    weight = loss.lf_weight(target, gamma=0.5, form=1)
    out = oracle.render(scene, [cam])
    _, g_view = loss.l1_loss_grad(out["views"][0], target, weight)
    dd, dsh = oracle.backward(scene, [cam], g_view.ravel())
    raw0, _ = oracle.voxel_colours(scene, [cam])
    tflat = np.asarray(target, np.float64).reshape(3, P)
    wflat = weight.reshape(P)
    rng = np.random.default_rng(251102513)
    hit = np.nonzero(out["wmax"] > 1e-3)[0]
    assert hit.shape[0] > 10000
    nb = (scene.sh_degree + 1) ** 2
    h = np.float32(1e-3)
    fd, an, tries = [], [], 0
    while len(fd) < 64 and tries < 300:
        tries += 1
        v = int(rng.choice(hit))
        if len(fd) < 32:
            arr, row = scene.density, int(rng.integers(0, 8))
        else:
            # SH rows over all degrees in turn: basis index i, channel ch
            i = int((len(fd) - 32) % nb)
            ch = int(rng.integers(0, 3))
            row = 3 * i + ch
            arr = scene.sh
            if abs(raw0[0, v, ch]) <= 2.0 * float(h):   # the clamp at zero is a kink
                continue
        pix = oracle.footprint_pixels(scene, [cam], np.array([v]))
        base = arr[row, v]
        vals, signs = [], []
        for sgn in (1, -1):
            arr[row, v] = np.float32(base + np.float32(sgn) * h)
            L, s = _pixel_loss(scene, cam, tflat, wflat, pix)
            vals.append(L)
            signs.append(s)
        hp = float(np.float32(base + h)) - float(base)
        hm = float(base) - float(np.float32(base - h))
        arr[row, v] = base
        if np.any(signs[0] != signs[1]):                    # an L1 residual changes sign
            continue
        fd.append((vals[0] - vals[1]) / (hp + hm))
        an.append(dd[row, v] if arr is scene.density else dsh[row, v])
    assert len(fd) == 64, (len(fd), tries)
    fd, an = np.array(fd), np.array(an)
    assert np.count_nonzero(an) > 48
    rel = np.linalg.norm(fd - an) / np.linalg.norm(an)
    assert rel < 1e-4, rel
