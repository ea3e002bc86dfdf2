"""Benchmark: fwd+bwd megapixels/s of the sparse-voxel tile rasterizer on one
MI355X, on the 1M-voxel SH3 workload with 8 ring views of uneven resolution.

One step = the whole hot path on one batch of views: projection + binning +
per-tile sort + composite forward with w_max, inverse-Sobel weights of the
targets, weighted L1 and its image gradient, composite backward, SH backward
and the depth-binned w_max quantile cutoff -- all views in one call per
phase, captured once in a HIP graph and replayed.  Inputs are synthetic
(seeded) and resident in HBM before timing starts.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd megapixels/s @1M voxels SH3 (batched vs single-view), % HBM roofline"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# algorithmic bytes per launch of the composite kernels, the per-unit figures
# of the hot-path byte model: per (tile, voxel) pair 4 B
# id + a 59 B record gather (forward), plus 11 reduced 4-byte gradients
# (backward: 107 B); per pixel 28 B (forward: rgb 12 + depth 4 + alpha 4 +
# saved state 8; backward: saved state 8 + rgb/depth/alpha gradients 20).
def composite_bytes(Q, P, which):
    if which == "composite_fwd":
        return 63 * Q + 28 * P
    return 107 * Q + 28 * P


PROFILE_MD = os.path.join(ROOT, "profiles", "composite_hbm_counters_ring1m.md")


def composite_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("paper_2511_02510_amd/csrc/k_raster.hip", "paper_2511_02510_amd/csrc/lv_common.h"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


VALU_MD = os.path.join(ROOT, "profiles", "composite_valu_ring1m.md")
VALU_PEAK = 256 * 4 * 2.4e9 / 4   # wave64 VALU instructions/s: 16-lane SIMDs, 4 per CU


def _profile_lines(path, name, kernel, tile, chunk):
    """Fields after `<name> <kernel>` of the committed counter summary line
    for these settings, or None (no such line, or the summary was taken on
    other composite kernel sources)."""
    try:
        with open(path) as fh:
            text = fh.read()
    except OSError:
        return None
    ok, found = False, None
    for line in text.splitlines():
        f = line.split()
        if f[:2] == ["composite_source_sha256_16", composite_source_hash()]:
            ok = True
        if len(f) >= 5 and f[0] == name and f[1] == kernel and f[3:5] == [f"tile={tile}", f"chunk={chunk}"]:
            found = f[2:]
    return found if ok else None


def counter_traffic(kernel, tile, chunk):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE
    summary, or None when it was taken on other kernel sources or settings."""
    t = _profile_lines(PROFILE_MD, "traffic_bytes_per_launch", "k_" + kernel, tile, chunk)
    return int(float(t[0])) if t else None


def counter_valu(kernel, tile, chunk, ms):
    """VALU issue of `kernel` from the committed counter summary: wave
    instructions per launch, issue rate over the launch time measured here
    against the chip's peak, and lane utilisation; None when stale."""
    t = _profile_lines(VALU_MD, "valu_instr_per_launch", "k_" + kernel, tile, chunk)
    if not t:
        return None
    inst = float(t[0])
    return {"wave_instr_per_launch": int(inst), "issue_frac": round(inst / (ms * 1e-3) / VALU_PEAK, 4),
            "peak_wave_instr_per_s": VALU_PEAK, "lane_util": float(t[4])}


# algorithmic bytes of the whole forward and backward (all phases), each
# byte the method must move counted once: N voxels, M visible (view, voxel) records, Q pairs, P pixels,
# K SH floats per voxel
def step_bytes(N, M, Q, P, K):
    b_fwd = N * (7 + 32 + 4 * K) + 4 * N + 20 * M + 91 * Q + 28 * P
    b_bwd = 107 * Q + 28 * P + 24 * M + (7 + 32 + 4 * K) * N
    return b_fwd, b_bwd


def training_step(lv, ctx, r, vox, frame, target, gamma, form, bufs, stream, side, quantile,
                  verify=False, overlap=True):
    """One step: forward, loss weight, L1 gradient, backward (+ depth quantile).
    With overlap, work that does not need the forward runs on `side` beside
    it: the loss weight (it needs only the target and gamma) and the depth
    quantile's binning (it needs only the geometry); the quantile's cutoff
    (it needs w_max) runs beside the L1 gradient.  Events join the two
    streams, also inside a captured graph.  The backward waits for the
    cutoff: run beside the backward, whose persistent workgroups fill every
    CU, the quantile's kernels slow it by more than they take alone.
    Without overlap everything runs in order on `stream`."""
    import torch
    rgb, depth, alpha, wmax, weight, lw_ws, loss, d_rgb, dd, dsh, nb, q_ws, tau, prune = bufs
    if not overlap:
        lv.lf_weight(ctx, frame, target, gamma, form, 1e-3, weight, lw_ws, stream=stream)
        r.forward(rgb, depth, alpha, wmax, stream=stream, verify=verify)
        lv.l1_grad(ctx, frame, rgb, target, weight, loss, d_rgb, stream=stream)
        r.backward(d_rgb, None, None, dd, dsh, stream=stream)
        if quantile:
            lv.depth_quantile(ctx, vox, frame, wmax, nb, 0.1, q_ws, tau, prune, stream=stream)
        return
    e0 = torch.cuda.Event()
    e0.record(stream)
    side.wait_event(e0)
    lv.lf_weight(ctx, frame, target, gamma, form, 1e-3, weight, lw_ws, stream=side)
    e_w = torch.cuda.Event()
    e_w.record(side)
    if quantile:
        lv.depth_bins(ctx, vox, frame, nb, q_ws, stream=side)
    r.forward(rgb, depth, alpha, wmax, stream=stream, verify=verify)
    e_f = torch.cuda.Event()
    e_f.record(stream)
    stream.wait_event(e_w)
    if quantile:
        side.wait_event(e_f)
        lv.depth_cutoff(ctx, vox, wmax, nb, 0.1, q_ws, tau, prune, stream=side)
        e_q = torch.cuda.Event()
        e_q.record(side)
    lv.l1_grad(ctx, frame, rgb, target, weight, loss, d_rgb, stream=stream)
    if quantile:
        stream.wait_event(e_q)
    r.backward(d_rgb, None, None, dd, dsh, stream=stream)


def measure_workload(lv, ctx, name, tile, chunk, chunk_bwd, reps, warmup, quantile, form, gamma):
    """Forward and whole-step MP/s of another named workload (graph replay)."""
    import torch
    import synth
    t0 = time.time()
    scene, cams, targets = synth.make_config(name)
    gen_s = time.time() - t0
    dev = torch.device("cuda", 0)
    vox = lv.Voxels.from_scene(scene, dev)
    frame = lv.Frame(cams, dev)
    P = frame.P
    target = torch.from_numpy(np.concatenate([t.ravel() for t in targets]).astype(np.float32)).to(dev)
    r = lv.Renderer(ctx, vox, frame, lv.settings(tile=tile, chunk=chunk, chunk_bwd=chunk_bwd))
    rgb, depth, alpha = r.new_outputs()
    wmax = torch.zeros(vox.n, device=dev)
    weight = torch.empty(P, device=dev)
    lw_ws = torch.empty(lv.lf_weight_workspace_size(frame.n_views), dtype=torch.uint8, device=dev)
    loss = torch.empty(frame.n_views, device=dev)
    d_rgb = torch.empty(3 * P, device=dev)
    dd, dsh = torch.empty_like(vox.density), torch.empty_like(vox.sh)
    nb = 16
    q_ws = torch.empty(lv.quantile_workspace_size(vox.n, nb), dtype=torch.uint8, device=dev)
    tau = torch.empty(nb, device=dev)
    prune = torch.empty(vox.n, dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream()
    side = torch.cuda.Stream()
    bufs = (rgb, depth, alpha, wmax, weight, lw_ws, loss, d_rgb, dd, dsh, nb, q_ws, tau, prune)

    def fwd(verify=False):
        r.forward(rgb, depth, alpha, wmax, stream=stream, verify=verify)

    def step(verify=False):
        training_step(lv, ctx, r, vox, frame, target, gamma, form, bufs, stream, side, quantile,
                      verify=verify)

    def timed(fn):
        with torch.cuda.stream(stream):
            fn(verify=True)
        torch.cuda.synchronize()
        lv.graph_begin(ctx, stream)
        fn()
        lv.graph_end(ctx, stream)
        for _ in range(warmup):
            lv.graph_launch(ctx, stream)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            lv.graph_launch(ctx, stream)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t) / reps
        lv.graph_reset(ctx)
        return ms

    fwd_ms = timed(fwd)
    Q, M = lv.pass_stats(ctx, vox, frame, r.st, r.saved, stream=stream)
    b_fwd, b_bwd = step_bytes(scene.n, M, Q, P, int(vox.sh.shape[0]))
    out = {"voxels": scene.n, "views": len(cams), "px": P, "pairs": Q, "records": M,
           "fwd_ms": round(fwd_ms, 4), "fwd_mp_s": round(P / fwd_ms / 1e3, 2),
           "fwd_bytes": int(b_fwd),
           "fwd_hbm_frac": round(b_fwd / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if name != "shell200k":          # that configuration is forward + w_max only
        step_ms = timed(step)
        out.update({"fwdbwd_ms": round(step_ms, 4), "fwdbwd_mp_s": round(P / step_ms / 1e3, 2),
                    "bwd_bytes": int(b_bwd),
                    "step_hbm_frac": round((b_fwd + b_bwd) / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "step": "fwd + lf_weight + l1 + bwd" + (" + depth quantile" if quantile else "")})
    log(f"[bench] {name}: {out} (scene generated in {gen_s:.1f} s)")
    del r, vox, frame, target
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ring1m")
    ap.add_argument("--tile", type=int, default=0, help="0 = autotune")
    ap.add_argument("--chunk", type=int, default=64, help="forward chunk (with --tile)")
    ap.add_argument("--chunk-bwd", type=int, default=0, help="backward chunk (0 = --chunk)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-views", type=int, default=8,
                    help="views of the workload the oracle baseline renders (8 = the whole step)")
    ap.add_argument("--profile-aux-steps", type=int, default=0,
                    help="run this many steps with the auxiliary channels and terms on one "
                         "stream and exit (for kernel traces)")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="if > 0: only run this many eager steps (for rocprofv3) and exit")
    ap.add_argument("--other-workloads", default="grid4k,shell200k,shell200k_train,hemi4m",
                    help="comma list of further workloads to report fwd and fwd+bwd MP/s for "
                         "(empty: none)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="if > 0: only copy this many MiB device-to-device 3 times (a kernel of "
                         "known traffic that calibrates the HBM byte counters) and exit")
    args = ap.parse_args()

    if args.copy_probe_mib > 0:
        import torch
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {4 * n} bytes x 3")
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): the library "
              "has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2511_02510_amd as lv

    t0 = time.time()
    scene, cams, targets = synth.make_config(args.workload)
    log(f"[bench] workload {args.workload}: N={scene.n} views={len(cams)} "
        f"sizes={[(c.width, c.height) for c in cams]} ({time.time() - t0:.1f}s)")
    dev = torch.device("cuda", 0)
    ctx = lv.Context(0)
    vox = lv.Voxels.from_scene(scene, dev)
    frame = lv.Frame(cams, dev)
    P = frame.P
    target = torch.from_numpy(np.concatenate([t.ravel() for t in targets]).astype(np.float32)).to(dev)

    if args.tile == 0:
        best, table = lv.autotune(ctx, vox, frame, reps=3)
        st = lv.settings(tile=best.tile, chunk=best.chunk, chunk_bwd=best.chunk_bwd,
                         pair_capacity=best.pair_capacity)
        log(f"[bench] autotune ms (forward, backward; tile 8/16/32 x chunk 64/128/256):\n"
            f"{np.round(table, 3)}")
    else:
        st = lv.settings(tile=args.tile, chunk=args.chunk, chunk_bwd=args.chunk_bwd)
    chunk_bwd = int(st.chunk_bwd) or int(st.chunk)
    log(f"[bench] settings tile={st.tile} chunk={st.chunk} chunk_bwd={chunk_bwd}")

    r = lv.Renderer(ctx, vox, frame, st)
    rgb, depth, alpha = r.new_outputs()
    wmax = torch.zeros(vox.n, device=dev)
    weight = torch.empty(P, device=dev)
    lw_ws = torch.empty(lv.lf_weight_workspace_size(frame.n_views), dtype=torch.uint8, device=dev)
    loss = torch.empty(frame.n_views, device=dev)
    d_rgb = torch.empty(3 * P, device=dev)
    d_density = torch.empty_like(vox.density)
    d_sh = torch.empty_like(vox.sh)
    n_bins, q = 16, 0.1
    q_ws = torch.empty(lv.quantile_workspace_size(vox.n, n_bins), dtype=torch.uint8, device=dev)
    tau = torch.empty(n_bins, device=dev)
    prune = torch.empty(vox.n, dtype=torch.uint8, device=dev)
    gamma = lv.gamma_schedule(0.5, 1.0)

    stream = torch.cuda.Stream()
    side = torch.cuda.Stream()   # both at the default priority
    bufs = (rgb, depth, alpha, wmax, weight, lw_ws, loss, d_rgb, d_density, d_sh, n_bins, q_ws, tau,
            prune)

    def step(verify=False, overlap=True):
        # q is 0.1 in both forms of the step
        training_step(lv, ctx, r, vox, frame, target, gamma, 0, bufs, stream, side, True,
                      verify=verify, overlap=overlap)

    with torch.cuda.stream(stream):
        step(verify=True, overlap=False)    # sizes the pair buffers exactly
    torch.cuda.synchronize()
    fits, Q = lv.check_overflow(ctx, vox, frame, r.st, r.saved, stream=stream)
    assert fits
    log(f"[bench] pairs Q={Q} capacity={r.st.pair_capacity}")

    # buffers of the step with the auxiliary channels and terms: forward with
    # the distortion, normal and median-depth channels, loss weight, L1, the
    # four auxiliary terms, one backward taking every channel's gradient
    dist_c, normal_c = torch.empty(P, device=dev), torch.empty(3 * P, device=dev)
    mdepth_c = torch.empty(P, device=dev)
    aloss = torch.empty(4 * len(cams), device=dev)
    ga_c, gd_c, gl_c = (torch.empty(P, device=dev) for _ in range(3))
    gn_c = torch.empty(3 * P, device=dev)

    def aux_step(verify=False):
        lv.lf_weight(ctx, frame, target, gamma, 0, 1e-3, weight, lw_ws, stream=stream)
        r.forward(rgb, depth, alpha, wmax, stream=stream, verify=verify, dist=dist_c,
                  normal=normal_c, mdepth=mdepth_c)
        lv.l1_grad(ctx, frame, rgb, target, weight, loss, d_rgb, stream=stream)
        lv.aux_loss(ctx, frame, depth, alpha, normal_c, dist_c, 0.01, 0.05, 1.0, aloss, ga_c,
                    gd_c, gn_c, gl_c, stream=stream, mdepth=mdepth_c, lam_nm=0.05)
        r.backward_aux(d_rgb, gd_c, ga_c, depth, gl_c, gn_c, d_density, d_sh, stream=stream)

    if args.profile_aux_steps > 0:
        aux_step(verify=True)
        for _ in range(args.profile_aux_steps):
            aux_step()
        torch.cuda.synchronize()
        log("[bench] auxiliary profile steps done")
        return

    if args.profile_steps > 0:
        for _ in range(args.profile_steps):
            step(overlap=False)     # one stream: kernel durations without neighbours
        torch.cuda.synchronize()
        log("[bench] profile steps done")
        return

    # ---- per-kernel timing (HIP events on the library's stream), eager
    lv.set_timing(ctx, True)
    lv.read_timings(ctx)
    for _ in range(max(3, args.steps // 2)):
        step(overlap=False)
    ph = lv.read_timings(ctx)
    lv.set_timing(ctx, False)
    phases = {k: (ms / max(c, 1)) for k, (ms, c) in ph.items()}
    log("[bench] phase ms/launch: " + ", ".join(f"{k} {v:.3f}" for k, v in phases.items()))

    # ---- graph capture of one whole step (loss weight and the depth
    # quantile's binning beside the forward, its cutoff beside the L1
    # gradient, on a second stream)
    lv.graph_begin(ctx, stream)
    step(overlap=True)
    lv.graph_end(ctx, stream)
    for _ in range(args.warmup):
        lv.graph_launch(ctx, stream)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        lv.graph_launch(ctx, stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_step = 1e3 * elapsed / args.steps
    value = P * args.steps / elapsed / 1e6
    log(f"[bench] graph step {ms_step:.3f} ms -> {value:.1f} MP/s fwd+bwd")

    # ---- forward-only graph
    lv.graph_reset(ctx)
    lv.graph_begin(ctx, stream)
    r.forward(rgb, depth, alpha, wmax, stream=stream, verify=False)
    lv.graph_end(ctx, stream)
    for _ in range(args.warmup):
        lv.graph_launch(ctx, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        lv.graph_launch(ctx, stream)
    torch.cuda.synchronize()
    fwd_ms = 1e3 * (time.perf_counter() - t1) / args.steps
    lv.graph_reset(ctx)

    # ---- single-view plain path: each view alone, eager, no graph
    single = []
    for v, c in enumerate(cams):
        f1 = lv.Frame([c], dev)
        r1 = lv.Renderer(ctx, vox, f1, lv.settings(tile=st.tile, chunk=st.chunk, chunk_bwd=chunk_bwd))
        o = r1.new_outputs()
        w1 = torch.empty(f1.P, device=dev)
        lw1 = torch.empty(lv.lf_weight_workspace_size(1), dtype=torch.uint8, device=dev)
        tg = target[3 * int(frame.off[v]):3 * int(frame.off[v + 1])]
        l1 = torch.empty(1, device=dev)
        g1 = torch.empty(3 * f1.P, device=dev)

        def one(verify=False):
            r1.forward(*o, wmax, stream=stream, verify=verify)
            lv.lf_weight(ctx, f1, tg, gamma, 0, 1e-3, w1, lw1, stream=stream)
            lv.l1_grad(ctx, f1, o[0], tg, w1, l1, g1, stream=stream)
            r1.backward(g1, None, None, d_density, d_sh, stream=stream)

        one(verify=True)
        for _ in range(2):
            one()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        reps = max(3, args.steps // 4)
        for _ in range(reps):
            one()
        torch.cuda.synchronize()
        single.append(1e3 * (time.perf_counter() - ts) / reps)
    log(f"[bench] single-view plain fwd+bwd ms: {np.round(single, 3).tolist()}")

    # ---- roofline of the dominant kernel
    dom = max(("composite_fwd", "composite_bwd"), key=lambda k: phases[k])
    alg = composite_bytes(Q, P, dom)
    achieved = alg / (phases[dom] * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
            "alg_bytes_per_launch": int(alg), "ms_per_launch": round(phases[dom], 4)}
    dom_chunk = chunk_bwd if dom == "composite_bwd" else int(st.chunk)
    roof["traffic"] = counter_traffic(dom, int(st.tile), dom_chunk)
    roof["valu"] = counter_valu(dom, int(st.tile), dom_chunk, phases[dom])
    fwd_alg = composite_bytes(Q, P, "composite_fwd")
    fwd_roof = fwd_alg / (phases["composite_fwd"] * 1e-3) / 1e9

    # ---- whole-forward and whole-step HBM fractions (all phases)
    _, M = lv.pass_stats(ctx, vox, frame, r.st, r.saved, stream=stream)
    b_fwd, b_bwd = step_bytes(scene.n, M, Q, P, int(vox.sh.shape[0]))
    hbm = {"records": M, "fwd_bytes": int(b_fwd), "bwd_bytes": int(b_bwd),
           "fwd_frac": round(b_fwd / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "step_frac": round((b_fwd + b_bwd) / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    log(f"[bench] whole-path HBM fractions {hbm}")

    # ---- pruning stability guards (the next row after the hot path): one
    # adaptation step on this workload's w_max, the cap binding
    gbins = torch.empty(vox.n, dtype=torch.uint8, device=dev)
    lv.depth_quantile(ctx, vox, frame, wmax, n_bins, 0.1, q_ws, tau, prune, gbins, stream=stream)
    gws = torch.empty(lv.guard_workspace_size(vox.n), dtype=torch.uint8, device=dev)
    ema = torch.empty(vox.n, device=dev)
    gstate = torch.empty(vox.n, dtype=torch.uint8, device=dev)
    gprune = torch.empty(vox.n, dtype=torch.uint8, device=dev)
    npr = torch.empty(1, dtype=torch.int32, device=dev)
    gp = lv.guard_params(alpha=0.5, cap_frac=0.01)
    gtimes = []
    for rep in range(max(5, args.steps // 2) + 2):
        with torch.cuda.stream(stream):
            ema.fill_(0.5)      # every voxel starts halfway: many candidates, the cap binds
            gstate.fill_(1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lv.prune_guard(ctx, vox, frame, wmax, gbins, tau, n_bins, gp, gws, ema, gstate, gprune, npr,
                       stream=stream)
        e1.record(stream)
        e1.synchronize()
        if rep >= 2:
            gtimes.append(e0.elapsed_time(e1))
    g_ms = float(np.median(gtimes))
    g_bytes = 23 * scene.n   # w_max, bin, ema, state, level, ijk read; ema, state, prune written
    guard = {"voxels": scene.n, "ms": round(g_ms, 4), "pruned": int(npr.cpu().numpy()[0]),
             "alg_bytes": int(g_bytes),
             "hbm_frac": round(g_bytes / (g_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    log(f"[bench] prune guard {guard}")

    # ---- priority-driven subdivision (the next row after the guards): the
    # footprint percentiles, the selection with w_max as usefulness, the split
    def gpu_ms(fn, reps):
        ts = []
        for rep in range(reps + 2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            if rep >= 2:
                ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    sws = torch.empty(lv.split_workspace_size(vox.n), dtype=torch.uint8, device=dev)
    zr = torch.empty(2, device=dev)
    ssplit = torch.empty(vox.n, dtype=torch.uint8, device=dev)
    nsp = torch.empty(1, dtype=torch.int32, device=dev)
    spp = lv.split_params()
    reps = max(5, args.steps // 2)
    t_range = gpu_ms(lambda: lv.footprint_range(ctx, vox, frame, sws, zr, stream=stream), reps)
    t_sel = gpu_ms(lambda: lv.subdivide_select(ctx, vox, frame, wmax, zr, spp, sws, ssplit, None, nsp,
                                               stream=stream), reps)
    n_split = int(nsp.cpu().numpy()[0])
    n_out = scene.n + 7 * n_split
    t_apply = gpu_ms(lambda: lv.subdivide_apply(ctx, vox, ssplit, n_out, sws, stream=stream), reps)
    per_voxel = 7 + 32 + 4 * int(vox.sh.shape[0])      # ijk + level, densities, SH
    subdiv = {"voxels": scene.n, "splits": n_split, "voxels_after": n_out,
           "range_ms": round(t_range, 4), "select_ms": round(t_sel, 4), "apply_ms": round(t_apply, 4),
           "apply_alg_bytes": int(per_voxel * (scene.n + n_out)),
           "apply_hbm_frac": round(per_voxel * (scene.n + n_out) / (t_apply * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    log(f"[bench] subdivision {subdiv}")

    # ---- the auxiliary channels and terms on this workload (the step built
    # above)
    aux_step(verify=True)
    torch.cuda.synchronize()
    lv.set_timing(ctx, True)
    lv.read_timings(ctx)
    for _ in range(max(3, args.steps // 2)):
        aux_step()
    aph = lv.read_timings(ctx)
    lv.set_timing(ctx, False)
    aphases = {k: (ms / max(c, 1)) for k, (ms, c) in aph.items()}
    # ten calls back to back per timed interval, so host-side gaps between
    # the event and the launch do not count
    t_aux_loss = gpu_ms(lambda: [lv.aux_loss(ctx, frame, depth, alpha, normal_c, dist_c, 0.01,
                                             0.05, 1.0, aloss, ga_c, gd_c, gn_c, gl_c,
                                             stream=stream, mdepth=mdepth_c, lam_nm=0.05)
                                 for _ in range(10)],
                        max(5, args.steps // 2)) / 10
    lv.graph_begin(ctx, stream)
    aux_step()
    lv.graph_end(ctx, stream)
    for _ in range(args.warmup):
        lv.graph_launch(ctx, stream)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for _ in range(args.steps):
        lv.graph_launch(ctx, stream)
    torch.cuda.synchronize()
    aux_ms = 1e3 * (time.perf_counter() - ta) / args.steps
    lv.graph_reset(ctx)
    aux = {"step": "fwd (+ distortion, normal, median depth) + lf_weight + l1 + 4 aux terms + "
                   "bwd (all channels)",
           "ms_per_step": round(aux_ms, 4), "mp_s": round(P / aux_ms / 1e3, 2),
           "composite_fwd_ms": round(aphases["composite_fwd"], 4),
           "composite_bwd_ms": round(aphases["composite_bwd"], 4),
           "aux_loss_ms": round(t_aux_loss, 4),
           "plain_composite_fwd_ms": round(phases["composite_fwd"], 4),
           "plain_composite_bwd_ms": round(phases["composite_bwd"], 4)}
    log(f"[bench] auxiliary channels and terms {aux}")

    # ---- the other workloads
    others = {}
    for name in [w for w in args.other_workloads.split(",") if w]:
        spec = {"grid4k": (False, 0, 0.5), "shell200k": (False, 1, 0.5),
                "shell200k_train": (False, 1, 0.5), "hemi4m": (True, 0, 0.5)}[name]
        others[name] = measure_workload(lv, ctx, name, int(st.tile), int(st.chunk), chunk_bwd,
                                        max(3, args.steps // 2), 2, *spec)

    # ---- CPU baseline: the oracle on a bounded sample (the first views)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        nv = max(1, min(args.cpu_sample_views, len(cams)))
        sub = cams[:nv]
        rng = np.random.default_rng(0)
        Ps = sum(c.npix for c in sub)
        g = rng.normal(0, 1e-3, 3 * Ps)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        tc = time.perf_counter()
        oracle.render(scene, sub, threads=threads)
        t_fwd = time.perf_counter() - tc
        oracle.backward(scene, sub, g, threads=threads)
        dt = time.perf_counter() - tc
        # one thread on an evenly spread 1/16 of the same pixels
        pix1 = np.arange(0, Ps, 16)
        t1 = time.perf_counter()
        oracle.render(scene, sub, pix_list=pix1, threads=1)
        oracle.backward(scene, sub, g, pix_list=pix1, threads=1)   # gradient of the listed pixels
        dt1 = time.perf_counter() - t1
        cpu_model = ""
        try:
            with open("/proc/cpuinfo") as fh:
                cpu_model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
        except OSError:
            pass
        cpu = {"value": round(Ps / dt / 1e6, 4), "unit": "MP/s", "cores": threads, "kind": "oracle",
               "sample": f"fwd+bwd of view(s) 0..{nv - 1} ({Ps} px) of the same workload, FP64, "
                         f"{dt:.1f} s",
               "fwd_value": round(Ps / t_fwd / 1e6, 4),
               "one_thread_value": round(pix1.shape[0] / dt1 / 1e6, 4),
               "one_thread_sample": f"fwd+bwd of every 16th pixel of the same views ({pix1.shape[0]} px), "
                                    f"{dt1:.1f} s",
               "cpu_model": cpu_model, "host_threads": os.cpu_count()}
        log(f"[bench] oracle {cpu}")

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "MP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {scene.n} voxels (octree levels 7-11, shell + 10% "
                               f"clutter), SH degree 3, {len(cams)} ring views "
                               f"{[(c.width, c.height) for c in cams]}, {P} px per step",
                   "tile": int(st.tile), "chunk": int(st.chunk), "chunk_bwd": chunk_bwd,
                   "pairs": int(Q),
                   "streams": "render and gradient on one stream; loss weight and the depth "
                              "quantile's binning beside the forward, its cutoff beside the L1 "
                              "gradient, on a second (one graph)"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "fwd_mp_s": round(P / fwd_ms / 1e3, 2),
        "fwd_ms": round(fwd_ms, 4),
        "fwd_composite_hbm_frac": round(fwd_roof / HBM_PEAK_GBS, 4),
        "per_view_ms_batched": round(ms_step / len(cams), 4),
        "single_view_plain_ms": [round(x, 4) for x in single],
        "phases_ms": {k: round(v, 4) for k, v in phases.items()},
        "whole_path_hbm": hbm,
        "other_workloads": others,
        "next_rows": {"prune_guard": guard, "subdivide": subdiv, "aux_terms": aux},
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
