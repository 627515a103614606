"""Stage-1 benchmark: 3DGStream NTC training iterations/s on one MI355X.

One step = one Stage-1 iteration on the workload `arc-300k-1352px` (300K
Gaussians with SH degree 3, 20 training views at 1352x1014 on a forward arc,
targets rendered from a seeded rigid-plus-sinusoidal motion of the scene):
NTC query at every mean, transform + render of one view, L1 + D-SSIM loss,
backward through renderer and NTC, Adam step.  Inputs are resident in HBM
before timing starts.  Also reported: render FPS of the held-out view with
and without the NTC, the FP32 direct-optimisation comparator's iterations/s,
per-kernel device times, the roofline position of the dominant kernel, and
the CPU oracle timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HERE = os.path.dirname(os.path.abspath(__file__))
METRIC = "Stage-1 train iters/s + render FPS, 300K Gaussians @1352x1014, vs FP32 direct"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="arc-300k-1352px")
    ap.add_argument("--precision", default="f16", choices=["f32", "f16", "bf16"])
    ap.add_argument("--sort-mode", default="depth_first", choices=["depth_first", "radix64"])
    ap.add_argument("--warmup-iters", type=int, default=3000, help="NTC warm-up (Eq. 7) iterations before timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-direct", action="store_true")
    ap.add_argument("--render-reps", type=int, default=50)
    ap.add_argument("--frame-reps", type=int, default=6,
                    help="frames of 150 iterations timed for s/frame (the first is a warm-up; 0 = skip)")
    ap.add_argument("--batch-views", type=int, default=4,
                    help="views per step of the multi-view batch variant (1 = skip it)")
    ap.add_argument("--other-precisions", default="f32,bf16",
                    help="NTC precisions also timed (comma-separated; empty = none)")
    ap.add_argument("--protocol", action="store_true",
                    help="only the equal-PSNR comparison, with full logs")
    ap.add_argument("--protocol-iters", type=int, default=1000, help="iterations per method in the protocol")
    ap.add_argument("--quality-workloads", default="arc-300k-1352px,surfaces-300k-1352px",
                    help="workloads of the equal-PSNR comparison (the benchmark workload first)")
    ap.add_argument("--no-quality", action="store_true")
    ap.add_argument("--stream", type=int, default=0,
                    help="instead of the timing run, stream this many frames of a capture-like sequence "
                         "(Stage 1 + bake + Stage 2 + four novel views per frame)")
    ap.add_argument("--stream-gaussians", type=int, default=500_000)
    ap.add_argument("--stream-size", default="1920x1080")
    ap.add_argument("--stream-views", type=int, default=15)
    ap.add_argument("--scale", action="store_true",
                    help="instead of the timing run: forward + backward of 1M Gaussians at 1920x1080, "
                         "with the memory the context holds")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB, a kernel of known traffic "
                         "for calibrating the HBM byte counters")
    return ap.parse_args()


def quality(args, workload, iters=150, max_iters=1000, seeds=(0, 1, 2)):
    """Equal-PSNR protocol on one workload (the benchmark's steps: up to
    `max_iters` iterations per method, held-out PSNR logged every 10): the
    FP16/BF16 NTC (warm-started by Eq. 7) and FP32 direct optimisation of
    per-Gaussian (dmu, dq), same renderer, loss and view order.  Reading (a):
    NTC's PSNR at `iters` iterations is P*; the direct optimiser's training
    time to its first logged point at or above P* - 0.1 dB, against NTC's
    time for `iters` iterations.  Reading (b): the level both reach, min(best
    NTC, best direct) - 0.1 dB, and each one's time to it.  Training time
    only (the once-per-scene warm-up is reported apart).  One run per view-
    order seed; mean and range over the seeds.  Also the NTC from its random
    initialisation ('w/o warm-up')."""
    import torch
    from paper_2403_01444_amd import gs3, synth, train
    g, cams, held, nxt = synth.workload(workload, seed=0)
    cfg = synth.NTCConfig()
    W = max(c.width for c in cams + held)
    H = max(c.height for c in cams + held)
    ctx = gs3.Context(g.n, 120_000_000, W, H, num_slots=1, sort_mode=args.sort_mode, ntc=cfg,
                      precision=args.precision)
    gg = gs3.GaussiansGPU.from_host(g)
    gg, perm = ctx.reorder(gg, cfg.aabb_min, cfg.inv_extent())
    gn = gs3.GaussiansGPU.from_host(nxt.subset(perm.cpu().numpy().astype(np.int64)))
    targets = [ctx.render(gn, c).clone() for c in cams]
    ht = ctx.render(gn, held[0]).clone()
    K, _ = ctx.debug_counts()
    ctx.ntc_init(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    train.warmup(ctx, torch.from_numpy(synth.warmup_points(gg.means.cpu().numpy(), cfg, 1)).cuda(),
                 args.warmup_iters)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    warm = ctx.ntc_save_state()
    ctx.ntc_init(0)
    cold = ctx.ntc_save_state()
    psnr_static = train.psnr(ctx.render(gg, held[0]), ht)
    img = ctx.empty(3, held[0].height, held[0].width)
    runs = []
    for seed in seeds:
        ctx.ntc_load_state(warm)
        st = train.Stage1NTC(ctx, gg, cams, targets, lam=0.2, seed=seed)
        ntc_log = train.logged_run(st.step, lambda: train.psnr(ctx.render(gg, held[0], *st.transform(), image=img),
                                                               ht), max_iters)
        d = train.Stage1Direct(ctx, gg, cams, targets, lam=0.2, seed=seed)
        direct_log = train.logged_run(d.step, lambda: train.psnr(ctx.render(gg, held[0], d.dmu, d.dq, image=img),
                                                                 ht), max_iters)
        ctx.ntc_load_state(cold)
        st_cold = train.Stage1NTC(ctx, gg, cams, targets, lam=0.2, seed=seed)
        cold_log = train.logged_run(st_cold.step,
                                    lambda: train.psnr(ctx.render(gg, held[0], *st_cold.transform(), image=img), ht),
                                    iters)
        del st, d, st_cold
        runs.append((train.equal_psnr(ntc_log, direct_log, iters), ntc_log, direct_log, cold_log))
    ctx.check_flags()
    ctx.close()

    def agg(key):
        v = [r[0][key] for r in runs]
        ok = [x for x in v if x is not None]
        if not ok:
            return {"mean": None, "min": None, "max": None, "runs": v}
        return {"mean": round(float(np.mean(ok)), 4), "min": round(float(min(ok)), 4),
                "max": round(float(max(ok)), 4), "runs": [None if x is None else round(x, 4) for x in v]}

    ntc_s = [r[0]["ntc_seconds"] for r in runs]
    dir_s = [r[0]["direct_seconds_to_match"] for r in runs]
    res = {"workload": workload, "pairs_per_view": int(K), "ntc_precision": args.precision, "seeds": list(seeds),
           "max_iters": max_iters, "psnr_untransformed": round(psnr_static, 3), "warmup_s": round(t_warm, 3),
           "warmup_iters": args.warmup_iters,
           "reading_a": {"p_star_ntc_psnr_at_iters": agg("ntc_psnr_at_iters"), "ntc_seconds": agg("ntc_seconds"),
                         "direct_seconds_to_p_star": agg("direct_seconds_to_match"),
                         "direct_iters_to_p_star": agg("direct_iters_to_match"),
                         "direct_never_reached": sum(x is None for x in dir_s),
                         "ntc_faster_runs": sum(1 for a, b in zip(ntc_s, dir_s) if b is None or a < b)},
           "reading_b": {"common_psnr": agg("common_psnr"), "ntc_seconds": agg("ntc_seconds_to_common"),
                         "direct_seconds": agg("direct_seconds_to_common")},
           "at_150": {"ntc_psnr": agg("ntc_psnr_at_iters"), "direct_psnr": agg("direct_psnr_at_same_iters"),
                      "ntc_seconds": agg("ntc_seconds"), "direct_seconds": agg("direct_seconds_at_same_iters")},
           "best": {"ntc_psnr": agg("ntc_best_psnr"), "direct_psnr": agg("direct_best_psnr")},
           "ntc_psnr": {str(i): round(float(np.mean([dict((a, c) for a, _, c in r[1])[i] for r in runs])), 3)
                        for i in (10, 20, 50, 100, 150, 300, 500, 1000) if i <= max_iters},
           "direct_psnr": {str(i): round(float(np.mean([dict((a, c) for a, _, c in r[2])[i] for r in runs])), 3)
                           for i in (10, 20, 50, 100, 150, 300, 500, 1000) if i <= max_iters},
           "ntc_without_warmup_psnr": {str(i): round(float(np.mean([dict((a, c) for a, _, c in r[3])[i]
                                                                   for r in runs])), 3)
                                       for i in (20, 50, iters)},
           "ntc_iters_per_s": round(float(np.mean([max_iters / r[1][-1][1] for r in runs])), 2),
           "direct_iters_per_s": round(float(np.mean([max_iters / r[2][-1][1] for r in runs])), 2)}
    if args.protocol:
        res["logs"] = [{"seed": sd, "ntc": [(i, round(t, 5), round(p, 4)) for i, t, p in r[1]],
                        "direct": [(i, round(t, 5), round(p, 4)) for i, t, p in r[2]],
                        "ntc_without_warmup": [(i, round(t, 5), round(p, 4)) for i, t, p in r[3]]}
                       for sd, r in zip(seeds, runs)]
    return res


def scale(args):
    """1M Gaussians (SH3) at 1920x1080 with a small transform: render and
    renderer backward timed; device memory of the context; the per-pixel
    state kept between them (8 B: final transmittance and last walked entry)
    against storing a transmittance per walked (pixel, entry) (4 B each; an
    upper bound of the per-contributor count)."""
    import torch
    from paper_2403_01444_amd import gs3, synth
    g = synth.make_gaussians(1_000_000, 3, 21)
    cam = synth.look_at_camera(1920, 1080)
    rng = np.random.default_rng(22)
    dmu = torch.from_numpy((rng.normal(size=(g.n, 3)) * 0.005).astype(np.float32)).cuda()
    dq = torch.from_numpy((np.array([1, 0, 0, 0]) + rng.normal(size=(g.n, 4)) * 0.02).astype(np.float32)).cuda()
    ctx = gs3.Context(g.n, 400_000_000, 1920, 1080, num_slots=1)
    gg = gs3.GaussiansGPU.from_host(g)
    img = ctx.render(gg, cam, dmu, dq)
    dimg = torch.full_like(img, 1e-7)
    grads = {"d_dmu": ctx.zeros(g.n, 3), "d_dq": ctx.zeros(g.n, 4)}
    for _ in range(2):
        ctx.render(gg, cam, dmu, dq, image=img)
        ctx.render_backward(dimg, grads)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_reset()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.render(gg, cam, dmu, dq, image=img)
        ctx.render_backward(dimg, grads)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    ctx.profile(False)
    kernels = {}
    for name in ("preprocess_fwd", "radix_pass", "bin_count", "bin_scatter", "blend_fwd", "blend_bwd",
                 "preprocess_bwd"):
        ms, cnt = ctx.profile_query(name)
        if cnt:
            kernels[name] = round(ms / cnt, 4)
    K, _ = ctx.debug_counts()
    T, last = ctx.debug_pixels(cam)
    walked = int(last.to(torch.int64).sum())
    print(json.dumps({"mode": "scale", "gaussians": g.n, "width": 1920, "height": 1080, "pairs": int(K),
                      "ms_forward_backward": round(1000 * dt, 3), "kernels_ms": kernels,
                      "context_bytes": ctx.workspace_bytes(),
                      "per_pixel_state_bytes": 8 * 1920 * 1080,
                      "stored_T_counterfactual_bytes": 4 * walked, "data": "synthetic"}))


def stream(args):
    """Streaming run: per frame Stage 1 (150 iterations), bake, Stage 2 (100
    iterations), four novel views; new objects appear at 1/3 and 2/3 of the
    sequence.  Prints one JSON line with per-frame and mean figures."""
    import torch
    from paper_2403_01444_amd import gs3, stream as st, synth
    W, H = (int(v) for v in args.stream_size.split("x"))
    cfg = synth.NTCConfig()
    sc = synth.surface_scene(args.stream_gaussians, 3, 0)
    cams = synth.arc_cameras(args.stream_views, W, H)
    novel = st.novel_cameras(W, H)
    cap = 100_000
    ctx = gs3.Context(sc.gaussians.n + cap + 2 * 2000, 120_000_000, W, H, ntc=cfg, precision=args.precision)
    g0 = gs3.GaussiansGPU.from_host(sc.gaussians)
    tr = st.StreamTrainer(ctx, g0, cams, novel, cfg, warmup_iters=args.warmup_iters, max_add=cap)
    frames = []
    new_at = (max(1, args.stream // 3), max(2, 2 * args.stream // 3))
    for f, gt in st.synthetic_sequence(sc, args.stream, 1, new_objects=new_at):
        gtg = gs3.GaussiansGPU.from_host(gt)
        targets = [ctx.render(gtg, c).clone() for c in cams]
        novel_t = [ctx.render(gtg, c).clone() for c in novel]
        r = tr.frame(f, targets, novel_t)
        frames.append(r)
        print(json.dumps({"frame": f, "stage1_s": round(r.stage1_s, 4), "stage2_s": round(r.stage2_s, 4),
                          "spawned": r.spawned, "additional": r.additional,
                          "psnr_stage1": round(r.psnr_stage1, 3), "psnr_stage2": round(r.psnr_stage2, 3),
                          "render_fps": round(r.render_fps, 1)}), file=sys.stderr, flush=True)
    mean = lambda k: float(np.mean([getattr(r, k) for r in frames]))
    print(json.dumps({
        "mode": "stream", "frames": len(frames), "gaussians": sc.gaussians.n, "width": W, "height": H,
        "training_views": len(cams), "novel_views": len(novel), "new_objects_at": list(new_at),
        "warmup_s": round(tr.warmup_s, 3),
        "s_per_frame": round(mean("stage1_s") + mean("stage2_s"), 4),
        "stage1_s": round(mean("stage1_s"), 4), "stage2_s": round(mean("stage2_s"), 4),
        "psnr_stage1": round(mean("psnr_stage1"), 3), "psnr_stage2": round(mean("psnr_stage2"), 3),
        "render_fps": round(mean("render_fps"), 1), "additional_mean": round(mean("additional"), 1),
        "ntc_precision": args.precision, "data": "synthetic"}))


# Per-unit algorithmic work of each kernel.  The blend kernels are bound by
# vector ALU work.  The reported count is about 25 operations per evaluated
# (pixel, tile-list entry) pair, where a tile evaluates 256 x its longest
# walk (the 16 x 16 pixels of a tile run in lockstep up to the last
# contributor of any of them): evaluated pairs = 256 x sum over tiles of the
# longest walk.  The build's own per-operation counts of the two kernels'
# formulas (29 forward, 71 backward per pixel's own walked entries: Eq. 4 and
# its adjoint, add / mul / compare / min / exp 1, fused multiply-add 2, the
# backward with the 9 adds into the Gaussian's gradient terms) are reported
# beside it, never as the roofline.
OPS_PER_EVALUATED_PAIR = 25
BLEND_FWD_FLOP = 29
BLEND_BWD_FLOP = 71
FP32_VECTOR_PEAK_TFLOPS = 157.3

# Algorithmic HBM bytes of the rasterizer (preprocess, prefix sum, keys, sort,
# ranges, both blends, preprocess backward) per unit: per Gaussian the
# preprocess reads 72 + 4S and writes 52 bytes, the scan moves 8, the
# accumulators are zeroed (36) and the preprocess backward reads 36 + 72 + 4S
# and writes 28; per pair 52 bytes (emit 12, one sort read and write 24,
# ranges 8, one list read in each blend 4 + 4); per pixel 20 written by the
# forward and 20 read by the backward.  (S: SH floats per Gaussian.)
RASTER_KERNELS = ("preprocess_fwd", "radix_pass", "bin_gather", "bin_count", "scan", "bin_scatter", "tile_ranges",
                  "tile_order", "blend_fwd", "blend_bwd", "preprocess_bwd")


def raster_bytes(n, K, P, S):
    return n * (72 + 4 * S + 52 + 8 + 36 + 36 + 72 + 4 * S + 28) + K * 52 + P * (20 + 20)


def algorithmic_work(name, st):
    """(bound, amount per step, unit) of the work the method itself needs
    (a kernel launched twice per step, like the two phases of the binning
    scatter and the forward blend, shares it between its launches)."""
    n, P, S = st["n"], st["pixels"], st["sh_floats"]
    if name in ("blend_fwd", "blend_bwd"):
        return "alu", 256 * st["walked"] * OPS_PER_EVALUATED_PAIR, "flop"
    if name == "preprocess_fwd":
        # read mean, quat, log-scale, opacity, SH, dmu, dq; write 48-byte record, key, rect, count
        return "hbm", n * (12 + 16 + 12 + 4 + 4 * S + 12 + 16 + 48 + 4 + 8 + 4), "byte"
    if name == "preprocess_bwd":
        # read the 36-byte gradient terms and the inputs again; write d_dmu, d_dq
        return "hbm", n * (36 + 12 + 16 + 12 + 4 + 4 * S + 12 + 16 + 12 + 16), "byte"
    if name == "ntc_fwd":
        return "hbm", n * (12 + 28) + st["table_bytes"], "byte"
    if name == "ntc_bwd":
        return "hbm", n * (12 + 28) + st["table_bytes"], "byte"
    if name == "ntc_scatter":
        # each contribution read once (entry weight and feature gradient), each table gradient written once
        return "hbm", st["contribs"] * (4 + 8) + 4 * st["table_entries"] * 2, "byte"
    if name == "loss":
        return "hbm", P * (12 + 12 + 12) + P * 36 * 2, "byte"
    if name == "bin_scatter":
        return "hbm", n * 16 + st["K"] * 4, "byte"
    if name == "bin_count":
        return "hbm", n * 16, "byte"
    return None


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc
    summary (FETCH_SIZE and WRITE_SIZE, scaled by what the counters read for
    a copy of known size), or None when there is no summary for this
    workload or kernel, or the kernel sources changed since it was taken."""
    import hashlib
    path = os.path.join(HERE, "profiles", f"stage1_step_{workload}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ": " in line and not line.startswith(" "):
            k, v = line.strip().split(": ", 1)
            kv[k] = v
    row = kv.get(f"traffic {kernel}")
    if row is None:
        return None
    h = hashlib.sha256()
    for f in ("paper_2403_01444_amd/csrc/raster.hip", "paper_2403_01444_amd/csrc/common.h"):
        h.update(open(os.path.join(HERE, f), "rb").read())
    if h.hexdigest() != kv.get("source_sha256"):
        return None
    fetch_kib, write_kib = (float(x) for x in row.split())
    return int((fetch_kib * float(kv["fetch_factor"]) + write_kib * float(kv["write_factor"])) * 1024)


def cpu_baseline(g, cam, target_np, params, cfg):
    """The oracle timed on one complete Stage-1 iteration of the workload:
    NTC forward on all N means (float64 numpy), render of one full training
    view, Eq. 6 loss, render adjoint (float64 C, OpenMP), NTC backward, Adam.
    The CPU threads are those of the C oracle (OpenMP); numpy parts run on
    its default BLAS threads."""
    from oracle import loss as oloss
    from oracle import ntc as ontc
    from oracle import optim as oopt
    from oracle import raster as orc
    spec = ontc.NTCSpec(cfg)
    t0 = time.perf_counter()
    dmu, dq, cache = ontc.forward(spec, params, g.means)
    dmu32, dq32 = dmu.astype(np.float32), dq.astype(np.float32)
    t1 = time.perf_counter()
    out = orc.render(g, cam, dmu32, dq32)
    L, dL = oloss.stage1_loss(out["image"], target_np.astype(np.float64), 0.2)
    rb = orc.render_backward(g, cam, dL, dmu32, dq32)
    t2 = time.perf_counter()
    grad = ontc.backward(spec, params, cache, rb["d_dmu"], rb["d_dq"])
    oopt.adam(params, grad, np.zeros_like(grad), np.zeros_like(grad), 1, 0.002, 0.9, 0.99, 1e-15)
    t3 = time.perf_counter()
    total = t3 - t0
    return {"value": round(1.0 / total, 6), "unit": "iters/s", "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"one complete Stage-1 iteration (all {g.n} means, one full {cam.width}x{cam.height} view); "
                      f"float64 oracle: NTC {t1 - t0 + t3 - t2:.1f}s, render+loss+adjoint {t2 - t1:.1f}s, "
                      f"total {total:.1f}s"}


def time_stage1(st, steps, warmup):
    """Stage-1 iterations per second of a Stage1NTC loop."""
    import torch
    for _ in range(warmup):
        st.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st.step()
    torch.cuda.synchronize()
    return steps / (time.perf_counter() - t0)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the Stage-1 step of one frame is a single-GPU job here); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2403_01444_amd import gs3, synth, train

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.protocol:
        print(json.dumps([quality(args, w, max_iters=args.protocol_iters)
                          for w in args.quality_workloads.split(",") if w]))
        return
    if args.stream:
        stream(args)
        return
    if args.scale:
        scale(args)
        return
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 18, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    g, cams, held, nxt = synth.workload(args.workload, seed=0)
    cfg = synth.NTCConfig()
    W = max(c.width for c in cams + held)
    H = max(c.height for c in cams + held)
    max_pairs = 120_000_000
    ctx = gs3.Context(g.n, max_pairs, W, H, num_slots=1, sort_mode=args.sort_mode, ntc=cfg,
                      precision=args.precision)
    gg = gs3.GaussiansGPU.from_host(g)
    gn = gs3.GaussiansGPU.from_host(nxt)
    targets = [ctx.render(gn, c).clone() for c in cams]
    held_t = [ctx.render(gn, c).clone() for c in held]
    ctx.check_flags()
    # per-frame setup: the frozen Gaussians in Morton order
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gg, order = ctx.reorder(gg, cfg.aabb_min, cfg.inv_extent())
    torch.cuda.synchronize()
    t_reorder = time.perf_counter() - t0

    # NTC warm-up (Eq. 7) on noise-augmented means, then Stage 1
    params0 = synth.ntc_init_params(cfg, 0)
    ctx.ntc_load(params0)
    wp = torch.from_numpy(synth.warmup_points(g.means, cfg, 1)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    train.warmup(ctx, wp, args.warmup_iters)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    params_warm = ctx.ntc_save()
    ctx.ntc_load(params_warm)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st1 = train.Stage1NTC(ctx, gg, cams, targets, lam=0.2)   # includes the per-frame NTC preparation
    torch.cuda.synchronize()
    t_prepare = time.perf_counter() - t0
    for _ in range(args.warmup):
        st1.step()
    torch.cuda.synchronize()
    ctx.check_flags()
    # per-kernel device times: every launch bracketed by HIP events, in a pass
    # of its own before the timed region
    ctx.profile(True)
    ctx.profile_reset()
    for _ in range(args.steps):
        st1.step()
    torch.cuda.synchronize()
    ctx.profile(False)
    kernels = {}
    for name in ("ntc_fwd", "preprocess_fwd", "radix_pass", "bin_count", "scan", "bin_gather", "bin_scatter", "tile_ranges", "tile_order",
                 "blend_fwd", "loss", "blend_bwd", "preprocess_bwd", "ntc_bwd", "ntc_scatter", "ntc_adam"):
        ms, cnt = ctx.profile_query(name)
        if cnt:
            kernels[name] = {"ms_per_launch": ms / cnt, "launches_per_step": cnt / args.steps}
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_launch"] * kernels[k]["launches_per_step"]) if kernels else None
    # the timed region: only the dominant kernel's launches carry events, and
    # its roofline uses their average duration
    ctx.profile_only(dom)
    ctx.profile(True)
    ctx.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st1.step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.profile(False)
    ctx.profile_only(None)
    ctx.check_flags()
    dom_ms = None
    if dom is not None:
        ms, cnt = ctx.profile_query(dom)
        dom_ms = ms / cnt
    iters_per_s = args.steps / elapsed
    free_b, total_b = torch.cuda.mem_get_info()
    mem = {"context_workspace_bytes": ctx.workspace_bytes(), "device_in_use_bytes": int(total_b - free_b),
           "torch_peak_allocated_bytes": int(torch.cuda.max_memory_allocated())}

    # pairs, walked list entries and per-pixel evaluations, averaged over the
    # training views with the final transform
    dmu_f, dq_f = st1.transform()
    Ks, walks, evals = [], [], []
    for cam in cams:
        ctx.render(gg, cam, dmu_f, dq_f)
        sc, wk = ctx.debug_sums()          # sum of n_contrib; sum over tiles of the longest walk
        walks.append(wk)
        evals.append(sc)
        Ks.append(ctx.debug_counts()[0])
    K0, walked, n_evals = int(np.mean(Ks)), int(np.mean(walks)), int(np.mean(evals))

    # s/frame: per-frame setup (Morton order of the frozen Gaussians, NTC
    # contribution lists) + 150 iterations from the warm-up parameters, the
    # median of 5 frames after one warm-up frame
    frame_s = []
    g_in = gs3.GaussiansGPU.from_host(g)
    for rep in range(args.frame_reps):
        ctx.ntc_load(params_warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g_f, _ = ctx.reorder(g_in, cfg.aabb_min, cfg.inv_extent())
        st_f = train.Stage1NTC(ctx, g_f, cams, targets, lam=0.2)
        for _ in range(150):
            st_f.step()
        torch.cuda.synchronize()
        if rep:
            frame_s.append(time.perf_counter() - t0)
        del st_f, g_f
    ctx.check_flags()
    ctx.ntc_load(params_warm)
    s_per_frame = float(np.median(frame_s)) if frame_s else None

    # render FPS on the held-out view: NTC query + transform + raster (and raster alone)
    hc = held[0]
    img = ctx.empty(3, hc.height, hc.width)
    dmu, dq = st1.dmu, st1.dq
    for _ in range(3):
        ctx.ntc_forward(gg.means, dmu, dq)
        ctx.render(gg, hc, dmu, dq, image=img)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.render_reps):
        ctx.ntc_forward(gg.means, dmu, dq)
        ctx.render(gg, hc, dmu, dq, image=img)
    torch.cuda.synchronize()
    fps = args.render_reps / (time.perf_counter() - t0)
    psnr_ntc = train.psnr(img, held_t[0])
    t0 = time.perf_counter()
    for _ in range(args.render_reps):
        ctx.render(gg, hc, image=img)
    torch.cuda.synchronize()
    fps_plain = args.render_reps / (time.perf_counter() - t0)

    # multi-view batch: several views per NTC query, NTC backward and Adam step
    multi_view = None
    if args.batch_views > 1:
        stb = train.Stage1NTC(ctx, gg, cams, targets, lam=0.2, views_per_step=args.batch_views)
        ips = time_stage1(stb, args.steps, args.warmup)
        multi_view = {"views_per_step": args.batch_views, "iters_per_s": round(ips, 3),
                      "views_per_s": round(ips * args.batch_views, 3)}
        del stb
        ctx.ntc_load(params_warm)

    # the same iteration with the NTC in the other precisions
    by_precision = {args.precision: round(iters_per_s, 3)}
    for prec in args.other_precisions.split(","):
        if not prec or prec == args.precision:
            continue
        c2 = gs3.Context(g.n, max_pairs, W, H, num_slots=1, sort_mode=args.sort_mode, ntc=cfg, precision=prec)
        c2.ntc_load(params_warm)
        by_precision[prec] = round(time_stage1(train.Stage1NTC(c2, gg, cams, targets, lam=0.2),
                                               args.steps, args.warmup), 3)
        c2.close()

    # FP32 direct optimisation comparator (same renderer and loss)
    direct = None
    if not args.no_direct:
        d = train.Stage1Direct(ctx, gg, cams, targets, lam=0.2)
        for _ in range(args.warmup):
            d.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            d.step()
        torch.cuda.synchronize()
        direct = args.steps / (time.perf_counter() - t0)

    # roofline of the dominant kernel (by device time per step)
    n_table_entries = cfg.num_table_params() // 2
    st = dict(n=g.n, pixels=cams[0].width * cams[0].height, walked=walked, evals=n_evals,
              sh_floats=3 * (g.sh_degree + 1) ** 2, K=K0, contribs=8 * cfg.levels * g.n,
              table_bytes=n_table_entries * 2 * (4 if args.precision == "f32" else 2),
              table_entries=n_table_entries)
    roof = None
    if dom is not None:
        w = algorithmic_work(dom, st)
        if w is not None:
            bound, amount, unit = w
            sec = dom_ms * kernels[dom]["launches_per_step"] * 1e-3
            if bound == "alu":
                ach, peak, u = amount / sec / 1e12, FP32_VECTOR_PEAK_TFLOPS, "TFLOP/s"
            else:
                ach, peak, u = amount / sec / 1e9, HBM_PEAK_GBS, "GB/s"
            roof = {"kernel": dom, "bound": bound, "achieved": round(ach, 3), "peak": peak, "unit": u,
                    "frac": round(ach / peak, 4), "traffic": measured_traffic(dom, args.workload),
                    "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                    "algorithmic_per_launch": int(amount),
                    "algorithmic_unit": unit, "ms_per_launch": round(dom_ms, 5)}
    if roof is not None and dom in ("blend_fwd", "blend_bwd"):
        per = BLEND_FWD_FLOP if dom == "blend_fwd" else BLEND_BWD_FLOP
        roof["count"] = (f"{OPS_PER_EVALUATED_PAIR} ops x 256 x {walked} (sum over tiles of the longest walk) "
                         f"evaluated pairs")
        roof["builder_op_count"] = {"ops_per_pixel_entry": per, "pixel_entries": n_evals,
                                    "tflops": round(per * n_evals / (dom_ms * 1e-3) / 1e12, 3),
                                    "frac": round(per * n_evals / (dom_ms * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS, 4)}
    r_ms = sum(kernels[k]["ms_per_launch"] * kernels[k]["launches_per_step"] for k in RASTER_KERNELS if k in kernels)
    r_bytes = raster_bytes(g.n, K0, cams[0].width * cams[0].height, 3 * (g.sh_degree + 1) ** 2)
    raster_hbm = {"kernels": list(RASTER_KERNELS), "ms_per_step": round(r_ms, 4), "algorithmic_bytes": int(r_bytes),
                  "achieved_gbs": round(r_bytes / (r_ms * 1e-3) / 1e9, 1),
                  "frac_of_8tbs": round(r_bytes / (r_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    all_roof = {}
    for k, v in kernels.items():
        w = algorithmic_work(k, st)
        if w is None:
            continue
        bound, amount, unit = w
        sec = v["ms_per_launch"] * v["launches_per_step"] * 1e-3
        all_roof[k] = (round(amount / sec / 1e12 / FP32_VECTOR_PEAK_TFLOPS, 4) if bound == "alu"
                       else round(amount / sec / 1e9 / HBM_PEAK_GBS, 4))

    # the NTC table gradient two ways on the same loop: the CSR gather over
    # the per-frame contribution lists (the step above) and per-point float
    # atomics into the table (token 0: no contribution lists, and the
    # backward gathers the encoding again)
    table_grad = None
    if "ntc_bwd" in kernels:
        tok = st1.token
        st1.token = 0
        for _ in range(args.warmup):
            st1.step()
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_reset()
        for _ in range(args.steps):
            st1.step()
        torch.cuda.synchronize()
        ctx.profile(False)
        st1.token = tok

        def per_step(name):
            ms, cnt = ctx.profile_query(name)
            return ms / args.steps if cnt else 0.0

        csr = {k: round(kernels[k]["ms_per_launch"] * kernels[k]["launches_per_step"], 4)
               for k in ("ntc_fwd", "ntc_bwd", "ntc_scatter") if k in kernels}
        atom = {k: round(per_step(k), 4) for k in ("ntc_fwd", "ntc_bwd")}
        table_grad = {"csr_gather_ms_per_step": csr, "csr_gather_backward_ms": round(csr["ntc_bwd"] +
                                                                                    csr.get("ntc_scatter", 0.0), 4),
                      "atomic_ms_per_step": atom, "atomic_backward_ms": atom["ntc_bwd"],
                      "used": "csr_gather"}
        ctx.ntc_load(params_warm)

    qual = None
    if not args.no_quality:
        del st1
        ctx.close()
        qual = [quality(args, w, max_iters=args.protocol_iters) for w in args.quality_workloads.split(",") if w]

    base = None
    if not args.no_cpu_baseline:
        g_ordered = g.subset(order.cpu().numpy().astype(np.int64))
        base = cpu_baseline(g_ordered, cams[0], targets[0].cpu().numpy(), params_warm, cfg)

    res = {
        "metric": METRIC, "value": round(iters_per_s, 3), "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1000.0 * elapsed / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": f"f32 raster + {args.precision} NTC",
        "data": "synthetic",
        "config": {"workload": args.workload, "gaussians": g.n, "sh_degree": g.sh_degree,
                   "width": cams[0].width, "height": cams[0].height, "views": len(cams),
                   "ntc_precision": args.precision, "sort_mode": args.sort_mode},
        "s_per_frame_150_iters": None if s_per_frame is None else round(s_per_frame, 4),
        "s_per_frame_runs": [round(x, 4) for x in frame_s],
        "s_per_frame_note": "per-frame setup (Morton order + NTC contribution lists) + 150 iterations, "
                            "median of 5 frames after 1 warm-up frame",
        "render_fps_with_ntc": round(fps, 2), "render_fps_without_ntc": round(fps_plain, 2),
        "direct_f32_iters_per_s": None if direct is None else round(direct, 3),
        "iters_per_s_by_ntc_precision": by_precision, "multi_view_batch": multi_view,
        "pairs_per_view": int(K0), "sum_n_contrib": n_evals, "walked_entries": walked,
        "evaluated_pairs": 256 * walked, "pixel_evals": n_evals,
        "device_memory": mem,
        "heldout_psnr_after_steps": round(psnr_ntc, 3),
        "warmup_s": round(t_warm, 3), "warmup_iters": args.warmup_iters, "frame_setup_s": round(t_prepare + t_reorder, 4),
        "kernels": {k: {kk: round(vv, 5) for kk, vv in v.items()} for k, v in kernels.items()},
        "roofline": roof, "roofline_frac_by_kernel": all_roof, "rasterizer_hbm": raster_hbm, "cpu_baseline": base,
        "ntc_table_gradient": table_grad, "equal_psnr": qual,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
