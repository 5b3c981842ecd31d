"""Benchmark of the batched Gaussian-splatting mapping step on one MI355X.

Workload: the batched keyframe window -- 1,000,000 Gaussians in an 8x8x3 m
room shell, 8 views at 1200x680 (f = 600) on a smooth trajectory, L1 colour
+ 0.1 L1 depth against renders from the unperturbed poses.  One step = the
whole hot path over all 8 views: projection, binning, compositing with the
fused loss, backward, pose reduction (and, for the mapping-iteration rate, the
Adam updates).  Every step is one hipGraph replay.

Prints one JSON line: fwd+bwd megapixels/s (the value), mapping iterations/s,
the per-view rate (the same kernels launched with V = 1 per view), the
roofline of the dominant kernel and the FP64 CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# launch shape timed by default: forward tiles 16x16 with 4 pixels per thread,
# bins 512x256, backward tiles 32x64 with 8 pixels per thread (the fastest in
# a sweep of shapes and bins on this workload; --tile auto tunes instead)
DEFAULT_LAUNCH = "16x16,4,512x256,32x64,8"

# published MI355X peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_VECTOR_TFLOPS = 157.3

# algorithmic FP32 operations per fragment (mul, add, compare-free; FMA = 2)
# forward: per candidate visited (offset 2, quadratic form 8, exp argument and
# exp 2, opacity product 1) = 13; per blended fragment (transmittance 2,
# weight 1, colour and depth accumulation 8) = +11; loss epilogue 16 per pixel
FWD_PER_VISIT, FWD_PER_BLEND, FWD_PER_PIXEL = 13, 11, 16
# backward: per candidate visited before the pixel's stop (13, as forward);
# per blended fragment: 1 - alpha and its reciprocal 2, transmittance 1,
# weight 1, colour/depth gradients 4, alpha gradient 16, suffix sums 8,
# opacity / sigma gradients 3, conic gradients 5, mean gradients 8 = +48
BWD_PER_VISIT, BWD_PER_BLEND = 13, 48


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_inputs(args):
    import numpy as np
    import torch
    import paper_2405_19614_amd as gs
    from synth import scenes
    s = scenes.c3(n=args.n, views=args.views, width=args.width, height=args.height)
    ctx = gs.Context(0)
    g = gs.Gaussians.from_scene(s, "cuda:0")
    poses = torch.tensor(np.asarray(s.poses, np.float32), device="cuda:0").reshape(s.V, 16).contiguous()
    poses_true = torch.tensor(np.asarray(s.poses_true, np.float32), device="cuda:0").reshape(s.V, 16).contiguous()
    # targets: renders from the unperturbed poses (input preparation, untimed)
    tc, td, _, _, _ = ctx.forward(g, s.cams, poses_true)
    return s, ctx, g, poses, tc, td


def timed_steps(step_fns, K, W):
    import torch
    for _ in range(W):
        for f in step_fns:
            f()
    torch.cuda.synchronize()
    # per-step event times (median) alongside the bracketed wall time
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        evs[k][0].record()
        for f in step_fns:
            f()
        evs[k][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) for a, b in evs]
    return wall * 1000.0 / K, statistics.median(per)


def cpu_baseline(s, views, min_seconds=10.0, max_reps=4):
    """FP64 oracle forward + L1 loss + backward on ``views`` of the workload,
    repeated until at least ``min_seconds`` of timed work (at most
    ``max_reps`` passes)."""
    import numpy as np
    from oracle import oracle as O
    og = O.Gaussians.from_scene(s)
    cams = [s.cams[v] for v in views]
    ptrue = [s.poses_true[v] for v in views]
    pest = [s.poses[v] for v in views]
    tgt = O.render_views(og, cams, ptrue)       # targets (untimed)
    reps, dt = 0, 0.0
    while reps < max_reps and (reps == 0 or dt < min_seconds):
        t0 = time.perf_counter()
        out = O.render_views(og, cams, pest)
        _, _, dC, dD = O.loss_and_upstream(cams, out, tgt["color"], tgt["depth"], 1.0, 0.1)
        O.backward_views(og, cams, pest, dC, dD, None)
        dt += time.perf_counter() - t0
        reps += 1
    px = sum(c.npix for c in cams)
    return px, reps, dt, O.num_threads()


def source_digest(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# sources that determine the compositing kernels' code
KERNEL_SOURCES = ["paper_2405_19614_amd/csrc/raster.hip", "paper_2405_19614_amd/csrc/gs_device.h",
                  "paper_2405_19614_amd/csrc/gs_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "composite_hbm_traffic_c3.md")


def measured_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed PMC summary, or
    None when the summary is missing or the kernel sources changed since."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    import re
    m = re.search(r"source digest[^`]*`([0-9a-f]+)`", text)
    if not m or m.group(1) != source_digest(KERNEL_SOURCES):
        return None
    m = re.search(r"^\| `?" + re.escape(kernel) + r"`? \|[^|]*\|[^|]*\|[^|]*\| ([0-9.]+) \|", text, re.M)
    return None if not m else float(m.group(1)) * 1e6


def copy_calibration(nbytes):
    """A plain device copy of ``nbytes`` (calibrates the PMC byte counters)."""
    import torch
    torch.cuda.set_device(0)
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "launches": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--views", type=int, default=8)
    ap.add_argument("--width", type=int, default=1200)
    ap.add_argument("--height", type=int, default=680)
    ap.add_argument("--tile", default=DEFAULT_LAUNCH,
                    help="auto | TWxTH,PPT,BWxBH[,BTWxBTH,BPPT] (tile, pixels per thread, bin[, backward tile, ppt]); "
                         "auto runs gs_autotune")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-views", type=int, default=8, help="views of the workload the CPU oracle runs")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="minimum timed CPU oracle work")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (PMC byte-counter calibration) and exit")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=5, help="eager steps timed per stage with HIP events")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library has no "
              "multi-GPU sharding", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    import torch
    import paper_2405_19614_amd as gs
    torch.cuda.set_device(0)
    log("[bench] building inputs")
    s, ctx, g, poses, tc, td = make_inputs(args)
    npix = s.npix
    if args.tile == "auto":
        tile, binsz = ctx.autotune(g, s.cams, poses, iters=2)
    else:
        # TWxTH,PPT,BWxBH[,BTWxBTH,BPPT]: forward tile, pixels per thread, bin[, backward tile and its ppt]
        vals = [int(x) for x in args.tile.lower().replace("x", ",").split(",")]
        tw, th, ppt, bw, bh = vals[:5]
        ctx.set_tile(tw, th, ppt)
        ctx.set_bin(bw, bh)
        if len(vals) == 8:
            ctx.set_bwd_shape(vals[5], vals[6], vals[7])
        tile, binsz = (tw, th), (bw, bh)
    btile = ctx.bwd_tile_choice if ctx.bwd_tile_choice != (0, 0) else tile
    ppt_f, ppt_b = ctx.ppt_choice(tile), ctx.ppt_choice(btile, True)
    log(f"[bench] tile {tile} x{ppt_f} bin {binsz} backward tile {btile} x{ppt_b}")
    base = dict(w_color=1.0, w_depth=0.1, w_reproj=0.0, tile=tile, bin=binsz, use_graph=True)

    # batched fwd+bwd (no update): the value
    st = gs.MappingStep(ctx, g, s.cams, poses, tc, td, gs.StepOptions(**base))
    st()
    torch.cuda.synchronize()
    status = st.status()
    if status["flags"]:
        raise RuntimeError(f"pair overflow: {status}")
    log(f"[bench] pairs {status['n_pairs']} visible {status['n_visible']} capacity {st.capacity}")
    ms, ms_med = timed_steps([st], args.steps, args.warmup)
    mpx = npix / (ms / 1000.0) / 1e6
    log(f"[bench] batched fwd+bwd: {ms:.3f} ms/step ({ms_med:.3f} median) -> {mpx:.1f} Mpx/s")

    # per-stage times and fragment counts (eager steps with HIP events)
    # (the counting pass runs the counting forward, so it is not timed)
    _, frag = st.profile(counts=True)
    stage_acc = {}
    for i in range(args.profile_steps):
        t, _ = st.profile(counts=False)
        for k, v in t.items():
            stage_acc.setdefault(k, []).append(v)
    stage_ms = {k: sum(v) / len(v) for k, v in stage_acc.items()}
    log(f"[bench] stages {json.dumps({k: round(v, 4) for k, v in stage_ms.items()})} frags {frag}")

    # mapping iterations (Adam on every Gaussian parameter)
    gm = gs.Gaussians(*(t.clone() for t in g.tensors()), g.sh_degree)
    stm = gs.MappingStep(ctx, gm, s.cams, poses.clone(), tc, td,
                         gs.StepOptions(update_gaussians=True, **base), capacity=st.capacity)
    ms_map, _ = timed_steps([stm], args.steps, args.warmup)
    iters = 1000.0 / ms_map
    log(f"[bench] mapping step: {ms_map:.3f} ms -> {iters:.2f} it/s")

    # the paper's mapping loss: (1 - zeta)(w4 L1_D + w5 L1_C) + zeta L_SSIM, Adam on the Gaussians
    gp = gs.Gaussians(*(t.clone() for t in g.tensors()), g.sh_degree)
    popts = dict(base)
    popts.update(gs.PAPER_MAPPING)
    stp = gs.MappingStep(ctx, gp, s.cams, poses.clone(), tc, td, gs.StepOptions(**popts), capacity=st.capacity)
    ms_paper, _ = timed_steps([stp], args.steps, args.warmup)
    t_paper, _ = stp.profile(counts=False)
    log(f"[bench] paper mapping loss (with SSIM): {ms_paper:.3f} ms -> {1000.0 / ms_paper:.2f} it/s; "
        f"ssim stage {t_paper.get('ssim', 0.0):.4f} ms")

    # per-view: the same kernels, V = 1 per launch sequence, V sequences per step
    per_view = None
    if not args.no_per_view:
        off = s.pix_offsets()
        pv_steps = []
        for v in range(s.V):
            pv_steps.append(gs.MappingStep(ctx, g, [s.cams[v]], poses[v:v + 1].clone(),
                                           tc[3 * off[v]:3 * off[v + 1]].contiguous(),
                                           td[off[v]:off[v + 1]].contiguous(),
                                           gs.StepOptions(**base)))
        ms_pv, _ = timed_steps(pv_steps, args.steps, args.warmup)
        per_view = npix / (ms_pv / 1000.0) / 1e6
        log(f"[bench] per-view fwd+bwd: {ms_pv:.3f} ms/step -> {per_view:.1f} Mpx/s")

    # roofline of the dominant kernel (compositing stages are one kernel each)
    dom = max(stage_ms, key=stage_ms.get)
    roof = None
    if frag is not None and dom in ("composite_bwd", "composite_fwd"):
        vis, blend = frag[0], frag[1]
        if dom == "composite_fwd":
            flops = FWD_PER_VISIT * vis + FWD_PER_BLEND * blend + FWD_PER_PIXEL * npix
        else:
            flops = BWD_PER_VISIT * vis + BWD_PER_BLEND * blend
        achieved = flops / (stage_ms[dom] / 1000.0) / 1e12
        kt = btile if dom == "composite_bwd" else tile
        kname = f"composite_{dom.split('_')[1]}_kernel<{kt[0]}, {kt[1]}, {ctx.ppt_choice(kt, dom == 'composite_bwd')}>"
        traffic = measured_traffic(kname)
        roof = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
                "traffic": None if traffic is None else int(traffic),
                "flops_per_launch": int(flops), "ms_per_launch": round(stage_ms[dom], 4),
                "traffic_GBs": None if traffic is None else round(traffic / (stage_ms[dom] / 1000.0) / 1e9, 1)}

    cpu = None
    if not args.no_cpu_baseline:
        views = list(range(min(args.cpu_views, s.V)))
        log(f"[bench] CPU oracle on views {views}")
        px, reps, dt, cores = cpu_baseline(s, views, args.cpu_seconds)
        cpu = {"value": round(px * reps / dt / 1e6, 5), "unit": "Mpx/s", "cores": cores, "kind": "oracle",
               "sample": f"FP64 oracle forward + L1 loss + backward of views {views} of the same workload "
                         f"({px} px), {reps} pass(es) in {dt:.1f} s"}

    out = {
        "metric": "fwd+bwd megapixels/s (batched, one graph replay per step); mapping iters/s and per-view rate "
                  "alongside",
        "value": round(mpx, 2),
        "unit": "Mpx/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched keyframe window: {s.n} Gaussians, room shell, {s.V} views "
                               f"{args.width}x{args.height}, f=600, L1 colour + 0.1 L1 depth",
                   "gaussians": s.n, "views": s.V, "width": args.width, "height": args.height,
                   "pixels_per_step": npix, "tile": f"{tile[0]}x{tile[1]}", "bin": f"{binsz[0]}x{binsz[1]}",
                   "bwd_tile": f"{btile[0]}x{btile[1]}", "pixels_per_thread": [ppt_f, ppt_b]},
        "mapping_iters_per_s": round(iters, 3),
        "ms_per_mapping_iter": round(ms_map, 4),
        "paper_mapping_loss_iters_per_s": round(1000.0 / ms_paper, 3),
        "ssim_stage_ms": round(t_paper.get("ssim", 0.0), 4),
        "per_view_mpx_s": None if per_view is None else round(per_view, 2),
        "batched_over_per_view": None if per_view is None else round(mpx / per_view, 3),
        "ms_per_step_median_events": round(ms_med, 4),
        "pairs": status["n_pairs"],
        "visible": status["n_visible"],
        "fragments": None if frag is None else {"visited": frag[0], "blended": frag[1], "entries_staged": frag[2],
                                                "list_entries": frag[3]},
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
