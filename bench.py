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

# Algorithmic cost models (documented in the design doc):
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
    return ap.parse_args()


def n_tiles_of(n_pix):
    return max(1, n_pix // 256)


def stage_bytes(n, n_front, n_vis, n_pairs, n_pix, n_views=1):
    """Algorithmic HBM bytes of each memory-bound stage for one launch."""
    return {
        # means of all (12) + scales, quats, opacity of those in front (32) + SH of
        # visible (192); writes: tiles + depth key of all (8) + record 48 + rect 8 of visible
        "project": 12 * n + 32 * n_front + 192 * n_vis + 8 * n * n_views + 56 * n_vis,
        # depth sort: 4 passes x (read key 4 + read key+val 8 + write 8) on all slots,
        # gather + scan (4 + 8 + 4 + 8), emission (8 per pair + 12 per visible),
        # tile sort passes x (4 + 8 + 8) per pair, ranges (4 per pair)
        "bin_sort": (4 * 20 * n * n_views + 24 * n * n_views + 8 * n_pairs + 12 * n_vis
                     + max(1, math.ceil(math.log2(max(2, n_tiles_of(n_pix))) / 8)) * 20 * n_pairs + 4 * n_pairs),
        # params of visible 236 + 2D grads 48 + outputs 236 + norm 4
        "project_bwd": 12 * n + 4 * n + (236 + 48) * n_vis + 236 * n + 4 * n,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path. "
              "How the path would shard is described in DESIGN.md.", file=sys.stderr)
        sys.exit(2)

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
        ed = depth / alpha.clamp_min(1e-10)
        loss = (rgb - tgt_rgb).abs().mean() + 0.5 * (ed - tgt_d).abs().mean()
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
        "serve_p50_ms": None,
        "serve_p99_ms": None,
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "workload_stats": {"visible": n_vis, "in_front": n_front, "pairs": P, "evals_fwd": e_fwd, "evals_bwd": e_bwd},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


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
    bins = oracle.bin_pairs(proj["rect"], proj["tiles"], keys, np.zeros(scene.n, np.int32), [sub])
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
