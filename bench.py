#!/usr/bin/env python
"""Benchmark of the differentiable rasterizer on one MI355X.

Workload (default): the 6M-Gaussian synthetic urban block seen from a
1920x1080 street-level camera with the anti-aliasing dilation and opacity
compensation, SH degree 3.  One step = projection + binning + compositing of
colour and depth + the loss (mean L1 on colour + 0.5 mean L1 on expected
depth) + the full backward to every parameter, i.e. one training iteration
without the optimiser.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
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

METRIC = "train fwd+bwd iters/s & render Mpix/s, 6M Gaussians 1080p; p50/p99 serve ms"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3     # MI355X vector FP32 (2 flops per FMA lane, dual issue)

# Algorithmic cost models:
# FP32 flops per compositing evaluation (an FMA counts 2, exp2 counts 1):
#   forward: dx, dy (2) + 3 products (3) + 2 FMA (4) + exp2 (1) + o'G (1)
#            + T(1 - a) (2) + a T (1) + 4 FMA blends (8)              = 22
#   backward (per entry before `last`): recompute (11) + rcp and T_i (2)
#            + weight (1) + dL/da (13) + colour/depth grads (4)
#            + d o', d power (2) + d mean (10) + d conic (7)
#            + recurrences (12) + |d mean| (0)                         = 62
FLOPS_FWD_EVAL = 22.0
FLOPS_BWD_EVAL = 62.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-crop", type=int, default=16, help="oracle baseline renders 1/crop of the pixels")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving trace")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests of the serving trace")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB device buffer 3 times (reference kernel for HBM byte counters)")
    return ap.parse_args()


def copy_probe(mib):
    """A plain device-to-device copy of known size: what the HBM byte counters
    read for it scales the counters of the rasterizer's kernels."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "copies": 3}))


def n_tiles_of(n_pix):
    return max(1, n_pix // 256)


def stage_bytes(n, n_front, n_vis, n_pairs, n_pix, n_views=1):
    """Algorithmic HBM bytes of each memory-bound stage for one launch
    (S = slots = n * views, V = visible slots, P = pairs)."""
    S = n * n_views
    tile_passes = max(1, math.ceil(math.log2(max(2, n_tiles_of(n_pix))) / 8))
    return {
        # means of all (12) + scales, quats, opacity of those in front (32) + SH row of
        # visible (192); writes: tiles + depth key of all (8) + record 64, rect 8, tile mask 8 of visible
        "project": 12 * n + 32 * n_front + 192 * n_vis + 8 * S + 80 * n_vis,
        # visible flags (tiles in, flag out) and their scan (12) over all slots; compaction
        # (tiles, position, key in; key, slot out of visible); depth sort of the visible, 4 passes
        # of (key 4 + key, value 8 in; 8 out); gather by depth rank (slot, tiles, rectangle,
        # mask in; tiles, rectangle, mask out: 44) and the scan of tiles (12); emission (8 per
        # pair, 20 per rank); tile sort passes of 20 per pair; ranges (4 per pair)
        "bin_sort": (8 * S + 12 * S + 12 * S + 8 * n_vis + 4 * 20 * n_vis + 44 * n_vis + 12 * n_vis
                     + 8 * n_pairs + 20 * n_vis + tile_passes * 20 * n_pairs + 4 * n_pairs),
        # tiles of all (4); params 236 + 2D grads 48 of visible; gradients 236 + norm 4 of all
        "project_bwd": 4 * S + (236 + 48) * n_vis + 236 * n + 4 * S,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    import torch
    import paper_2507_23006_amd as gs
    import synthetic as S

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    gs.load()
    dev = torch.device("cuda:0")
    t_gen = time.time()
    scene = S.scene_c3(seed=0)
    cam = S.camera_c3(seed=2)
    cams = [cam]
    H, W = cam.height, cam.width
    tgt_rgb = torch.from_numpy(S.target_rgb(H, W, seed=1)).to(dev).view(-1, 3)
    tgt_d = torch.from_numpy(S.target_depth(H, W, seed=1, lo=20.0, hi=45.0)).to(dev).view(-1)
    params = [torch.from_numpy(a).to(dev).requires_grad_(True) for a in scene.param_arrays()]
    opts = gs.RenderOptions(sh_degree=3, dilation=0.3, aa=True, absgrad=False)
    print(f"# workload ready in {time.time() - t_gen:.1f} s", file=sys.stderr, flush=True)

    stats = gs.RenderStats()

    def step():
        for p in params:
            p.grad = None
        rgb, depth, alpha = gs.rasterize(*params, cams, opts, stats)
        loss = gs.l1_depth_loss(rgb, depth, alpha, tgt_rgb, tgt_d, 0.5)
        loss.backward()
        return loss

    # stage timing with stream events
    marks = []

    def hook(name):
        ev = torch.cuda.Event(enable_timing=True)
        ev.record()
        marks.append((name, ev))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    stage_ms = {}
    gs.set_stage_hook(hook)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        marks.append(("start", _ev(torch)))
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gs.set_stage_hook(None)
    prev = None
    for name, ev in marks:
        if prev is not None and name != "start":
            stage_ms[name] = stage_ms.get(name, 0.0) + prev.elapsed_time(ev)
        prev = ev
    for k in stage_ms:
        stage_ms[k] /= args.steps
    # the interval ending at bwd_begin is the loss (torch ops between the two passes)
    if "bwd_begin" in stage_ms:
        stage_ms["loss"] = stage_ms.pop("bwd_begin")
    ms_step = (t1 - t0) * 1000.0 / args.steps

    # forward-only render rate
    with torch.no_grad():
        pd = [p.detach() for p in params]
        for _ in range(3):
            proj = gs.project(*pd, cams, opts)
            pv, rg, P = gs.bin_sort(proj, cams, scene.n)
            gs.render_fwd(proj, pv, rg, cams, opts)
        torch.cuda.synchronize()
        r0 = time.perf_counter()
        for _ in range(args.steps):
            proj = gs.project(*pd, cams, opts)
            pv, rg, P = gs.bin_sort(proj, cams, scene.n)
            out = gs.render_fwd(proj, pv, rg, cams, opts)
        torch.cuda.synchronize()
        r1 = time.perf_counter()
        ms_fwd = (r1 - r0) * 1000.0 / args.steps
        # workload statistics for the cost models (outside the timed regions)
        n_front = int((proj.depth_key.view(torch.int32) != -1).sum().item())
        tiles = proj.tiles
        n_vis = int((tiles > 0).sum().item())
        counts = gs.render_count(proj, pv, rg, cams).to(torch.int64).sum(0).tolist()
        e_fwd, e_bwd = int(counts[0]), int(counts[1])
    npix = W * H

    # roofline of the dominant stage
    stage_flops = {"render_fwd": FLOPS_FWD_EVAL * e_fwd, "composite_bwd": FLOPS_BWD_EVAL * e_bwd}
    dom = max((k for k in stage_ms if k != "loss"), key=stage_ms.get)
    roof = None
    if dom in stage_flops:
        ach = stage_flops[dom] / (stage_ms[dom] * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": dom, "achieved": round(ach, 3), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / FP32_PEAK_TFLOPS, 4), "traffic": None}
    else:
        b = stage_bytes(scene.n, n_front, n_vis, P, npix).get(dom)
        if b:
            ach = b / (stage_ms[dom] * 1e-3) / 1e9
            roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None}

    nxt = next_rows_bench(gs, torch, scene.n, W, H, dev, max(5, args.steps))

    # HBM fraction of every memory-bound stage, ALU fraction of compositing
    sb = stage_bytes(scene.n, n_front, n_vis, P, npix)
    stage_roof = {}
    for k, b in sb.items():
        if k in stage_ms:
            gbs = b / (stage_ms[k] * 1e-3) / 1e9
            stage_roof[k] = {"bound": "hbm", "bytes": int(b), "GB_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    for k, f in stage_flops.items():
        if k in stage_ms:
            tf = f / (stage_ms[k] * 1e-3) / 1e12
            stage_roof[k] = {"bound": "alu", "flops": int(f), "TFLOP_s": round(tf, 2),
                             "frac": round(tf / FP32_PEAK_TFLOPS, 4)}

    serve = None
    if not args.no_serve:
        del params, stats, proj, pv, rg, out
        serve = serve_bench(gs, S, torch, scene, opts, args.serve_requests)

    if roof is not None:
        roof["traffic"] = counted_traffic(roof["kernel"])

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(scene, cam, args.cpu_crop)

    rec = {
        "metric": METRIC,
        "value": round(1000.0 / ms_step, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "urban block: 6M Gaussians (70% ground, 30% facades of 200 boxes), "
                               "1920x1080 street-level camera, AA dilation 0.3 + compensation, SH3; "
                               "step = fwd + L1(rgb) + 0.5 L1(expected depth) + bwd to all parameters",
                   "n_gaussians": scene.n, "width": W, "height": H, "views": 1},
        "render_mpix_s": round(npix / (ms_fwd * 1e-3) / 1e6, 1),
        "render_ms": round(ms_fwd, 3),
        "serve_p50_ms": serve["served"]["p50_ms"] if serve else None,
        "serve_p99_ms": serve["served"]["p99_ms"] if serve else None,
        "serve": serve,
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "workload_stats": {"visible": n_vis, "in_front": n_front, "pairs": P, "evals_fwd": e_fwd, "evals_bwd": e_bwd},
        "roofline": roof,
        "stage_roofline": stage_roof,
        "cpu_baseline": cpu,
        "next_rows": nxt,
    }
    print(json.dumps(rec), flush=True)


# Algorithmic HBM bytes per unit of the kernels measured beside the step
APP_FWD_BYTES = 64 + 16            # per Gaussian: embedding in, offsets out
APP_BWD_BYTES = 64 + 16 + 16 + 64  # embedding, offsets and their gradient in; embedding gradient out
APP_FWD_MFMA, APP_BWD_MFMA = 64, 104          # v_mfma_f32_16x16x4_f32 per 64 Gaussians
MFMA_F32_FLOPS = 16 * 16 * 4 * 2
# D-SSIM per pixel (3 channels, float32): forward reads x, y and writes 3
# partials; backward reads the partials, x and y and writes dx
DSSIM_BYTES = (12 + 12 + 36) + (36 + 12 + 12 + 12)


# per Gaussian, one view: tiles + statistic read, sum and count read and written
DENS_ACC_BYTES = 4 + 4 + 8 + 8
# scales, opacity and rate read; filtered scales and opacity written
FILTER_FWD_BYTES = 12 + 4 + 4 + 12 + 4


class _Ctx:
    """Stand-in autograd context for timing a Function's forward alone."""

    def save_for_backward(self, *a):
        pass


def S_cam_ring(k):
    import synthetic as S
    import numpy as np
    eye = (120.0 * np.cos(k * 0.4), 120.0 * np.sin(k * 0.4), 1.7)
    return S.Camera(1371.1, 1371.1, 960.0, 540.0, S.look_at(eye, (0.0, 0.0, 1.7), up=(0, 0, 1)), 1920, 1080)


def next_rows_bench(gs, torch, n, W, H, dev, reps):
    """Appearance MLP (forward, backward) over the scene's n Gaussians and
    D-SSIM (value + gradient) over the W x H image, timed with events on the
    stream the library launches on; HBM fraction of the algorithmic bytes."""
    g = torch.Generator(device="cpu").manual_seed(5)
    gemb = torch.randn(n, 16, generator=g).to(dev)
    iemb = torch.randn(32, generator=g).to(dev)
    p = gs.AppearanceParams.init(dev, seed=6)
    dy = torch.randn(n, 4, generator=g).to(dev)
    d_reg = torch.ones(1, device=dev)

    def timed(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        a, b = _ev(torch), None
        for _ in range(reps):
            fn()
        b = _ev(torch)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    ms_f = timed(lambda: gs.appearance_mlp_fwd(gemb, iemb, p.w1, p.b1, p.w2, p.b2, 0.1))
    off, _ = gs.appearance_mlp_fwd(gemb, iemb, p.w1, p.b1, p.w2, p.b2, 0.1)
    ms_b = timed(lambda: gs.appearance_mlp_bwd(gemb, iemb, p.w1, p.b1, p.w2, p.b2, off, dy, d_reg, 0.1))
    # densification bookkeeping over one step's statistics and the 3D filter
    D = gs.densify
    st = D.DensifyStats(n, dev)
    tiles = (torch.rand(n, generator=g) < 0.16).to(torch.int32).to(dev)
    gn = (torch.rand(1, n, generator=g) * 6e-4).to(dev)
    ms_acc = timed(lambda: D.accumulate(st, tiles, grad_norm=gn))
    box = (-25.0, -25.0, -5.0), (25.0, 25.0, 45.0)
    means = (torch.rand(3, n, generator=g) * 300 - 150).to(dev)
    scl = torch.exp(torch.randn(3, n, generator=g) * 0.7 - 2.5).to(dev)
    opac = torch.rand(n, generator=g).to(dev)
    st.accum.copy_((torch.rand(n, generator=g) * 1e-3).to(dev))
    st.count.fill_(1)
    prm = D.DensifyParams(box[0], box[1], tau_min=2e-4, eta=4.0, d_max=50.0, budget=n + n // 50)
    ms_sel = timed(lambda: D.select(st, means, scl, opac, prm))
    cams16 = [S_cam_ring(k) for k in range(16)]
    ms_rate = timed(lambda: D.filter3d_rate(means, cams16))
    rate = D.filter3d_rate(means, cams16)
    ms_ff = timed(lambda: D.Filter3D.forward(_Ctx(), scl, opac, rate, 0.45))
    del st, tiles, gn, means, opac, rate
    img = torch.rand(H, W, 3, generator=g).to(dev)
    tgt = torch.rand(H, W, 3, generator=g).to(dev)
    ms_s = timed(lambda: gs.dssim_loss(img, tgt, 0.2))
    del gemb, dy, off

    def hbm(nbytes, ms):
        gbs = nbytes / (ms * 1e-3) / 1e9
        return {"achieved_GB_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}

    def mfma(n_mfma, ms):
        tf = n * n_mfma / 64 * MFMA_F32_FLOPS / (ms * 1e-3) / 1e12
        return {"achieved_TFLOP_s": round(tf, 2), "peak": 157.3, "frac": round(tf / 157.3, 4)}

    return {
        "appearance_mlp": {"n_gaussians": n, "fwd_ms": round(ms_f, 4), "bwd_ms": round(ms_b, 4),
                           "fwd_hbm": hbm(n * APP_FWD_BYTES, ms_f), "bwd_hbm": hbm(n * APP_BWD_BYTES, ms_b),
                           "fwd_mfma_f32": mfma(APP_FWD_MFMA, ms_f), "bwd_mfma_f32": mfma(APP_BWD_MFMA, ms_b)},
        "dssim": {"pixels": W * H, "ms": round(ms_s, 4), "hbm": hbm(W * H * DSSIM_BYTES, ms_s)},
        "densify": {"n_gaussians": n, "accumulate_ms": round(ms_acc, 4),
                    "accumulate_hbm": hbm(n * DENS_ACC_BYTES, ms_acc), "select_ms": round(ms_sel, 4),
                    "filter3d_rate_16cams_ms": round(ms_rate, 4), "filter3d_rate_hbm": hbm(n * 16, ms_rate),
                    "filter3d_fwd_ms": round(ms_ff, 4), "filter3d_fwd_hbm": hbm(n * FILTER_FWD_BYTES, ms_ff)},
    }


STAGE_KERNEL = {"render_fwd": "k_render_fwd", "composite_bwd": "k_render_bwd", "project": "k_project_fwd",
                "project_bwd": "k_project_bwd"}


def counted_traffic(stage):
    """HBM bytes per launch of the stage's kernel from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE scaled by a plain
    device copy), or None when the summary is missing or the compositing
    source has changed since the counters were taken."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "counters_urban6M_1080p.md")
    src = os.path.join(root, "paper_2507_23006_amd", "csrc", "render.hip")
    try:
        line = next(l for l in open(path) if l.strip().startswith("COUNTERS "))
        rec = json.loads(line.strip()[len("COUNTERS "):])
        if rec["render_hip_sha256"] != hashlib.sha256(open(src, "rb").read()).hexdigest():
            return None
        k = rec["kernels"][STAGE_KERNEL[stage]]
        return int(k["read_bytes"] + k["write_bytes"])
    except (OSError, StopIteration, KeyError, ValueError):
        return None


def serve_bench(gs, S, torch, fine, opts, n_requests):
    """Open-loop serving trace on the level-of-detail stand-in of the urban
    block: levels of 1M, 3M and 6M Gaussians resident in HBM, 30 m render-time
    partitions, thresholds (30, 60, inf) m; Poisson arrivals at 150 req/s,
    resolutions 640x360 / 1280x720 / 1920x1080 and budgets 1M / 3M / 6M
    drawn uniformly.  Run on the same trace: "plain" (one request per
    launch, one stream, FIFO) and "served" (continuous batching of up to 8
    views, two worker streams), then both again with every request arriving
    at once ("_burst": the saturated throughput).  Latency = completion -
    scheduled arrival."""
    t_gen = time.time()
    lod = S.lod_scene_c4(fine)
    sc, offsets = lod.combined()
    params = [torch.from_numpy(a).cuda() for a in sc.param_arrays()]
    table = gs.LodTable(lod.part_min, lod.part_max, offsets, lod.counts, lod.thresholds,
                        3.0 * float(sc.scales.max()))
    trace = S.serve_trace_c4(n_requests=n_requests)
    npx = [r["camera"].width * r["camera"].height for r in trace]
    flat = torch.empty(3 * sum(npx), dtype=torch.float32, device="cuda")
    outs, off = [], 0
    for r, k in zip(trace, npx):
        outs.append(flat[3 * off:3 * (off + k)].view(r["camera"].height, r["camera"].width, 3))
        off += k
    print(f"# serving scene ready in {time.time() - t_gen:.1f} s ({sc.n} Gaussians in {len(lod.levels)} levels, "
          f"{lod.counts.shape[1]} partitions)", file=sys.stderr, flush=True)
    modes = {
        "plain": gs.ServeConfig(max_views_per_batch=1, n_streams=1, slot_capacity=6_000_000,
                                pair_capacity=48_000_000, pixel_capacity=1 << 21, queue_capacity=n_requests),
        "served": gs.ServeConfig(max_views_per_batch=8, n_streams=2, slot_capacity=24_000_000,
                                 pair_capacity=96_000_000, pixel_capacity=1 << 24, queue_capacity=n_requests),
    }
    res = {}
    # the trace as scheduled, then the same requests all at once (saturation)
    runs = [(name, cfg, False) for name, cfg in modes.items()] + [(name + "_burst", cfg, True)
                                                                  for name, cfg in modes.items()]
    for name, cfg, burst in runs:
        srv = gs.Server(params, table, opts, cfg)
        t0 = srv.now() + 0.5
        for r, o in zip(trace, outs):
            srv.submit(r["camera"], r["budget"], o, t0 + (0.0 if burst else r["t"]))
        n_done, n_fail, views, t_print = 0, 0, 0, time.time()
        while n_done < len(trace):
            for c in srv.poll(max_items=512, timeout_us=200_000):
                n_done += 1
                n_fail += c["status"] != 0
            if time.time() - t_print > 5.0:
                print(f"# {name}: {n_done}/{len(trace)} served", file=sys.stderr, flush=True)
                t_print = time.time()
        st = srv.stats()
        srv.close()
        res[name] = {"p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                     "mean_ms": round(st["mean_ms"], 3), "max_ms": round(st["max_ms"], 3),
                     "req_per_s": round(st["req_per_s"], 2), "mpix_per_s": round(st["mpix_per_s"], 1),
                     "mean_batch_views": round(st["mean_batch_views"], 3), "batches": st["batches"],
                     "completed": st["completed"], "failed": st["failed"]}
        print(f"# {name}: {res[name]}", file=sys.stderr, flush=True)
    res["trace"] = (f"{len(trace)} requests, Poisson {len(trace) / trace[-1]['t']:.0f} req/s over "
                    f"{trace[-1]['t']:.1f} s, offered {sum(npx) / trace[-1]['t'] / 1e6:.0f} Mpix/s")
    return res


def _ev(torch):
    ev = torch.cuda.Event(enable_timing=True)
    ev.record()
    return ev


def cpu_baseline(scene, cam, crop: int):
    """The FP64 oracle on a bounded sample of the same workload: every
    Gaussian is projected and back-projected for a camera that sees a
    centred 1/crop of the image (same pose and focal length, tile-aligned),
    and binning, compositing and its backward run on that crop.  The
    full-image time is extrapolated as projection + projection backward +
    crop * (binning + compositing + compositing backward)."""
    import oracle
    import synthetic as S
    cw = max(16, int(round(cam.width / math.sqrt(crop) / 16)) * 16)
    ch = max(16, int(round(cam.height / math.sqrt(crop) / 16)) * 16)
    x0 = ((cam.width - cw) // 2) // 16 * 16
    y0 = ((cam.height - ch) // 2) // 16 * 16
    sub = S.Camera(cam.fx, cam.fy, cam.cx - x0, cam.cy - y0, cam.viewmat, cw, ch)
    frac = (cw * ch) / (cam.width * cam.height)
    opt = dict(sh_degree=3, aa=True)
    t = {}
    a = time.perf_counter()
    proj = oracle.project(scene, sub, **opt)
    t["project"] = time.perf_counter() - a
    a = time.perf_counter()
    keys = oracle.depth_key(proj["depth"])
    bins = oracle.bin_pairs(proj["rect"], proj["tiles"], keys, np.zeros(scene.n, np.int32), [sub], mask=proj["mask"])
    t["bin"] = time.perf_counter() - a
    twod = oracle._twod([proj])
    a = time.perf_counter()
    img = oracle.render_view(sub, opt, 0, twod, bins["pair_slot"], bins["ranges"], guard_eps=None)
    t["render"] = time.perf_counter() - a
    g = (np.sign(img["rgb"]) / img["rgb"].size, np.zeros_like(img["depth"]), np.zeros_like(img["alpha"]))
    a = time.perf_counter()
    d2 = np.zeros((scene.n, 10))
    oracle.render_bwd_view(sub, opt, 0, twod, bins["pair_slot"], bins["ranges"], *g, d2, None)
    t["render_bwd"] = time.perf_counter() - a
    grads = {"means": np.zeros((3, scene.n)), "scales": np.zeros((3, scene.n)), "quats": np.zeros((4, scene.n)),
             "opacities": np.zeros(scene.n), "sh": np.zeros((16, 3, scene.n))}
    a = time.perf_counter()
    oracle.project_bwd(scene, sub, opt, d2, grads)
    t["project_bwd"] = time.perf_counter() - a
    full = t["project"] + t["project_bwd"] + (t["bin"] + t["render"] + t["render_bwd"]) / frac
    return {"value": round(1.0 / full, 5), "unit": "iters/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"all {scene.n} Gaussians projected and back-projected (FP64) for a centred {cw}x{ch} crop "
                      f"camera ({frac:.3f} of the pixels); binning, compositing and its backward on that crop, "
                      f"scaled by 1/{frac:.3f}",
            "seconds": {k: round(v, 2) for k, v in t.items()}, "extrapolated_s_per_iter": round(full, 2)}


if __name__ == "__main__":
    main()
