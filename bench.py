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

# Algorithmic cost models per unit of work, on each kernel's own duration:
# * compositing forward: an evaluation is one (pixel, list entry whose alpha
#   box holds the pixel centre) up to the pixel's stop; ~14 VALU operations
#   and one exp (a quarter-rate transcendental, 4 issue slots) = 18 issue
#   slots per evaluation;
# * compositing backward: an evaluation is one (pixel, box-covered entry) up
#   to the pixel's last composited entry; ~40 VALU operations, one exp and
#   one reciprocal = 42 operations per evaluation;
# * projection: 16 B per Gaussian (mean, plus the tile count written) and
#   272 B per visible Gaussian (the other 224 B of parameters read, 48 B of
#   record written);
# * binning: 172 B per pair (12 B emitted, 8 B histogram read, 24 B per
#   8-bit pass of a 45-bit (tile, depth) key sort -- 6 passes --, 8 B range
#   read), whatever the design does;
# * projection backward: 536 B per visible Gaussian (236 B parameters, 40 B
#   2D gradients and 16 B saved values read; 236 B gradients and 8 B
#   statistics written).
# ALU work is reported in TFLOP/s of those operations against the 157.3
# TFLOP/s FP32 vector peak (packed, FMA = 2), and as a fraction of the issue
# ceiling of 256 CUs x 64 lanes x 2.4 GHz = 39.3e12 lane operations/s (the
# non-packed rate this build runs at).
OPS_FWD_EVAL = 18.0
OPS_BWD_EVAL = 42.0
ISSUE_PEAK = 256 * 64 * 2.4e9
BIN_BYTES_PER_PAIR = 172.0
PROJ_BYTES_ALL, PROJ_BYTES_VIS = 16.0, 272.0
PROJ_BWD_BYTES_VIS = 536.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-crop", type=int, default=16, help="oracle baseline renders 1/crop of the pixels")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving trace")
    ap.add_argument("--no-configs", action="store_true", help="skip the C1, C2 and C5 lines")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving trace (for profiling) and print its record")
    ap.add_argument("--config", choices=("C1", "C2", "C5"), default=None,
                    help="time only this configuration's step (for profiling) and print its record")
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


def copy_rate(torch, mib=1024, reps=5):
    """Achievable HBM rate: a plain 1 GiB device-to-device copy timed with
    events, (bytes read + bytes written) / median time, GB/s."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    del src, dst
    return 2.0 * n * 4 / (pct(times, 50) * 1e-3) / 1e9


def pct(xs, q):
    """q-quantile (linear interpolation) of a list of step times."""
    return float(np.percentile(np.asarray(xs, np.float64), q))


def step_times(torch, step, steps, warmup):
    """W untimed steps, then K steps bracketed by a synchronisation on both
    sides; each step also between two events on the current stream.
    Returns (wall ms per step over the K steps, per-step event ms)."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        evs.append(_ev(torch))
        step()
    evs.append(_ev(torch))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
    return (t1 - t0) * 1000.0 / steps, per


def summary(per):
    return {"median": round(pct(per, 50), 4), "p10": round(pct(per, 10), 4), "p90": round(pct(per, 90), 4),
            "mean": round(float(np.mean(per)), 4)}


def in_front(torch, params, cams):
    """Gaussians whose view depth lies in [near, far] of some view."""
    means = params[0].detach()
    hit = torch.zeros(means.shape[1], dtype=torch.bool, device=means.device)
    for c in cams:
        vm = torch.tensor(np.asarray(c.viewmat, np.float32), device=means.device)
        z = vm[2, :3] @ means + vm[2, 3]
        hit |= (z >= c.near) & (z <= c.far)
    return int(hit.sum().item())


def kernel_roofline(name, ms, n, n_vis, P, e_fwd, e_bwd):
    """The per-unit model of one timed kernel over its own average launch
    duration `ms`."""
    t = ms * 1e-3
    if name in ("k_render_fwd", "k_render_bwd"):
        ops = (OPS_FWD_EVAL * e_fwd) if name == "k_render_fwd" else (OPS_BWD_EVAL * e_bwd)
        evals = e_fwd if name == "k_render_fwd" else e_bwd
        ach = ops / t / 1e12
        return {"bound": "alu", "kernel": name, "achieved": round(ach, 3), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / FP32_PEAK_TFLOPS, 4),
                "issue_frac": round(ops / t / ISSUE_PEAK, 4), "evals_per_s": round(evals / t, 1),
                "model": f"{OPS_FWD_EVAL if name == 'k_render_fwd' else OPS_BWD_EVAL:.0f} operations x {evals} "
                         f"evaluations per launch", "launch_ms": round(ms, 4)}
    if name == "k_project_fwd":
        b = PROJ_BYTES_ALL * n + PROJ_BYTES_VIS * n_vis
        model = f"16 B x {n} Gaussians + 272 B x {n_vis} visible"
    elif name == "bin_sort":
        b = BIN_BYTES_PER_PAIR * P
        model = f"172 B x {P} pairs"
    else:
        b = PROJ_BWD_BYTES_VIS * n_vis
        model = f"536 B x {n_vis} visible"
    ach = b / t / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "bytes": int(b), "model": model, "launch_ms": round(ms, 4)}


def train_config(gs, torch, S, scene, cams, opts, tgt, steps, warmup, depth_term=True):
    """One training step (projection, binning, compositing, loss, full
    backward) on the given views: step times, forward-only render times,
    pairs and visible counts."""
    dev = torch.device("cuda:0")
    params = [torch.from_numpy(a).to(dev).requires_grad_(True) for a in scene.param_arrays()]
    stats = gs.RenderStats()
    tgt_rgb, tgt_d = tgt

    def step():
        for p in params:
            p.grad = None
        rgb, depth, alpha = gs.rasterize(*params, cams, opts, stats)
        loss = gs.l1_depth_loss(rgb, depth, alpha, tgt_rgb, tgt_d if depth_term else None, 0.5)
        loss.backward()

    wall, per = step_times(torch, step, steps, warmup)
    pd = [p.detach() for p in params]

    def fwd():
        proj = gs.project(*pd, cams, opts)
        pv, rg, P = gs.bin_sort(proj, cams, scene.n, sync=False)
        gs.render_fwd(proj, pv, rg, cams, opts)
        return P

    with torch.no_grad():
        _, per_f = step_times(torch, fwd, steps, warmup)
        assert not fwd().overflowed()
        proj = gs.project(*pd, cams, opts)
        pv, rg, P = gs.bin_sort(proj, cams, scene.n)
        n_vis = int((proj.tiles > 0).sum().item())
    npix = sum(c.width * c.height for c in cams)
    med, med_f = pct(per, 50), pct(per_f, 50)
    out = {"iters_per_s": round(1000.0 / med, 2), "step_ms": summary(per), "wall_ms_per_step": round(wall, 4),
           "render_mpix_s": round(npix / (med_f * 1e-3) / 1e6, 1), "render_ms": summary(per_f),
           "gaussians": scene.n, "views": len(cams), "pixels": npix, "visible_slots": n_vis, "pairs": int(P)}
    del params, stats, pd, proj, pv, rg
    torch.cuda.synchronize()
    return out


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
    if args.config:
        rec = other_configs(gs, torch, S, args, not args.no_cpu, only=args.config)[args.config]
        print(json.dumps({"configuration": args.config, **rec}), flush=True)
        return
    dev = torch.device("cuda:0")
    t_gen = time.time()
    scene = S.scene_c3(seed=0)
    if args.serve_only:
        opts = gs.RenderOptions(sh_degree=3, dilation=0.3, aa=True, absgrad=False)
        serve = serve_bench(gs, S, torch, scene, opts, args.serve_requests, with_cpu=False)
        print(json.dumps({"serving": serve}), flush=True)
        return
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

    # the timed steps alone: W untimed steps, then K steps between two
    # synchronisations (one event per step boundary for the percentiles)
    ms_step, per_step = step_times(torch, step, args.steps, args.warmup)

    # then, outside the timed region, stage times from stream events between
    # the library calls and the library's own events around each main
    # kernel, over a separate run of at most 20 steps, each read out (and
    # its events freed) before the next: many recorded events kept alive
    # make the runtime stall now and then
    n_inst = min(args.steps, 20)
    marks = []

    def hook(name):
        marks.append((name, _ev(torch)))

    gs.set_stage_hook(hook)
    gs.kernel_timing(True)
    torch.cuda.synchronize()
    stage_ms, k_tot, k_cnt = {}, {}, {}
    for _ in range(n_inst):
        marks.clear()
        marks.append(("start", _ev(torch)))
        step()
        torch.cuda.synchronize()
        prev = None
        for name, ev in marks:
            if prev is not None and name != "start":
                stage_ms[name] = stage_ms.get(name, 0.0) + prev.elapsed_time(ev)
            prev = ev
        for k in gs.rasterizer.KERNELS_TIMED:
            tot, cnt = gs.kernel_timing_read(k)
            k_tot[k] = k_tot.get(k, 0.0) + tot
            k_cnt[k] = k_cnt.get(k, 0) + cnt
    gs.set_stage_hook(None)
    gs.kernel_timing(False)
    marks.clear()
    kernel_ms = {k: k_tot[k] / k_cnt[k] for k in k_tot if k_cnt[k]}
    for k in stage_ms:
        stage_ms[k] /= n_inst
    # the interval ending at bwd_begin is the loss (torch ops between the two passes)
    if "bwd_begin" in stage_ms:
        stage_ms["loss"] = stage_ms.pop("bwd_begin")

    # forward-only render rate
    with torch.no_grad():
        pd = [p.detach() for p in params]

        def fwd():
            proj = gs.project(*pd, cams, opts)
            pv, rg, P = gs.bin_sort(proj, cams, scene.n, sync=False)
            gs.render_fwd(proj, pv, rg, cams, opts)
            return P

        _, per_fwd = step_times(torch, fwd, args.steps, args.warmup)
        assert not fwd().overflowed()
        ms_fwd = pct(per_fwd, 50)
        # workload statistics for the cost models (outside the timed regions)
        proj = gs.project(*pd, cams, opts)
        pv, rg, P = gs.bin_sort(proj, cams, scene.n)
        out = gs.render_fwd(proj, pv, rg, cams, opts)
        n_front = in_front(torch, params, cams)
        n_vis = int((proj.tiles > 0).sum().item())
        counts = gs.render_count(proj, pv, rg, cams).to(torch.int64).sum(0).tolist()
        e_fwd, e_bwd = int(counts[0]), int(counts[1])
    npix = W * H

    # every timed kernel against its model; the roofline object is the
    # longest-running one
    kroof = {k: kernel_roofline(k, ms, scene.n, n_vis, P, e_fwd, e_bwd) for k, ms in kernel_ms.items()}
    # the HBM-bound ones also against what a plain device copy achieves
    hbm_copy = copy_rate(torch)
    for r in kroof.values():
        if r["bound"] == "hbm":
            r["frac_of_copy"] = round(r["achieved"] / hbm_copy, 4)
    dom = max(kernel_ms, key=kernel_ms.get) if kernel_ms else None
    roof = dict(kroof[dom]) if dom else None

    nxt = next_rows_bench(gs, torch, scene.n, W, H, dev, max(5, args.steps))

    serve = None
    if not args.no_serve:
        del params, stats, proj, pv, rg, out
        serve = serve_bench(gs, S, torch, scene, opts, args.serve_requests, with_cpu=not args.no_cpu)

    if roof is not None:
        roof["traffic"] = counted_traffic(roof["kernel"])

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(scene, [cam], args.cpu_crop)

    configs = None
    if not args.no_configs:
        configs = other_configs(gs, torch, S, args, not args.no_cpu)

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
        "step_ms": summary(per_step),
        "iters_per_s_median": round(1000.0 / pct(per_step, 50), 3),
        "render_mpix_s": round(npix / (ms_fwd * 1e-3) / 1e6, 1),
        "render_ms": summary(per_fwd),
        "serve_p50_ms": serve["served"]["p50_ms"] if serve else None,
        "serve_p99_ms": serve["served"]["p99_ms"] if serve else None,
        "serve": serve,
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "kernel_ms": {k: round(v, 4) for k, v in kernel_ms.items()},
        "workload_stats": {"visible": n_vis, "in_front": n_front, "pairs": P, "evals_fwd": e_fwd, "evals_bwd": e_bwd},
        "roofline": roof,
        "kernel_roofline": kroof,
        "hbm_copy_GB_s": round(hbm_copy, 1),
        "cpu_baseline": cpu,
        "configs": configs,
        "next_rows": nxt,
    }
    print(json.dumps(rec), flush=True)


def other_configs(gs, torch, S, args, with_cpu, only=None):
    """C1 (4096 Gaussians, 160x120), C2 (1M, 1600x1066) and C5 (12M, eight
    views, 25.57 Mpix per launch): step times on the GPU beside the oracle
    on the host (C1 whole, C2 and C5 on a cropped sample)."""
    dev = torch.device("cuda:0")
    out = {}
    specs = [
        ("C1", lambda: (S.scene_c1(), [S.camera_c1()]), False, False, 1),
        ("C2", lambda: (S.scene_c2(seed=0), [S.camera_c2()]), False, True, 16),
        ("C5", lambda: (S.scene_urban(12_000_000, 400, seed=0), S.cameras_c5()), True, True, 64),
    ]
    for name, make, aa, depth_term, crop in specs:
        if only and name != only:
            continue
        t = time.time()
        scene, cams = make()
        tgt_rgb = torch.cat([torch.from_numpy(S.target_rgb(c.height, c.width, seed=1)).view(-1, 3) for c in cams]).to(dev)
        tgt_d = torch.cat([torch.from_numpy(S.target_depth(c.height, c.width, seed=1)).view(-1) for c in cams]).to(dev)
        opts = gs.RenderOptions(sh_degree=3, dilation=0.3, aa=aa)
        rec = train_config(gs, torch, S, scene, cams, opts, (tgt_rgb, tgt_d), args.steps, args.warmup, depth_term)
        if with_cpu:
            rec["cpu_baseline"] = cpu_baseline(scene, cams, crop, aa=aa, repeats=5 if crop == 1 else 1)
        out[name] = rec
        print(f"# {name}: {rec['iters_per_s']} iters/s, {rec['render_mpix_s']} Mpix/s ({time.time() - t:.1f} s)",
              file=sys.stderr, flush=True)
        del scene, tgt_rgb, tgt_d
    return out


# Algorithmic HBM bytes per unit of the kernels measured beside the step
APP_FWD_BYTES = 64 + 16            # per Gaussian: embedding in, offsets out
APP_BWD_BYTES = 64 + 16 + 16 + 64  # embedding, offsets and their gradient in; embedding gradient out
# algorithmic flops per Gaussian (the image-embedding half of the first
# layer is one bias per image): forward 16x32 + 32x4 products, backward dh,
# dW2, dW1 (Gaussian half) and dx
APP_FWD_FLOPS = 2 * (16 * 32 + 32 * 4)
APP_BWD_FLOPS = 2 * (32 * 4 + 32 * 4 + 16 * 32 + 16 * 32)
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

    def mfma(flops, ms):
        tf = n * flops / (ms * 1e-3) / 1e12
        return {"achieved_TFLOP_s": round(tf, 2), "peak": 157.3, "frac": round(tf / 157.3, 4),
                "flops_per_gaussian": flops}

    return {
        "appearance_mlp": {"n_gaussians": n, "fwd_ms": round(ms_f, 4), "bwd_ms": round(ms_b, 4),
                           "fwd_hbm": hbm(n * APP_FWD_BYTES, ms_f), "bwd_hbm": hbm(n * APP_BWD_BYTES, ms_b),
                           "fwd_mfma_f32": mfma(APP_FWD_FLOPS, ms_f), "bwd_mfma_f32": mfma(APP_BWD_FLOPS, ms_b)},
        "dssim": {"pixels": W * H, "ms": round(ms_s, 4), "hbm": hbm(W * H * DSSIM_BYTES, ms_s)},
        "densify": {"n_gaussians": n, "accumulate_ms": round(ms_acc, 4),
                    "accumulate_hbm": hbm(n * DENS_ACC_BYTES, ms_acc), "select_ms": round(ms_sel, 4),
                    "filter3d_rate_16cams_ms": round(ms_rate, 4), "filter3d_rate_hbm": hbm(n * 16, ms_rate),
                    "filter3d_fwd_ms": round(ms_ff, 4), "filter3d_fwd_hbm": hbm(n * FILTER_FWD_BYTES, ms_ff)},
    }


KERNEL_SOURCE = {"k_render_fwd": "render.hip", "k_render_bwd": "render.hip", "k_project_fwd": "project.hip",
                 "k_project_bwd": "project_bwd.hip"}


def counted_traffic(kernel):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain device copy), or
    None when the summary is missing or the kernel's source has changed since
    the counters were taken."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "counters_urban6M_1080p.md")
    try:
        src = os.path.join(root, "paper_2507_23006_amd", "csrc", KERNEL_SOURCE[kernel])
        line = next(l for l in open(path) if l.strip().startswith("COUNTERS "))
        rec = json.loads(line.strip()[len("COUNTERS "):])
        if rec["sources_sha256"][KERNEL_SOURCE[kernel]] != hashlib.sha256(open(src, "rb").read()).hexdigest():
            return None
        k = rec["kernels"][kernel]
        return int(k["read_bytes"] + k["write_bytes"])
    except (OSError, StopIteration, KeyError, ValueError):
        return None


def serve_modes(gs, n_requests):
    """Server configurations of the serving trace: "plain" (one request per
    launch, one worker, one batch in flight: FIFO) and "served" (continuous
    batching of up to 8 views admitted by estimated pairs, one worker with two
    batches in flight, so the next batch's projection and binning overlap the
    current compositing; a second worker measured no faster)."""
    return {
        "plain": gs.ServeConfig(max_views_per_batch=1, n_streams=1, pipeline_depth=1, slot_capacity=6_000_000,
                                pair_capacity=48_000_000, pixel_capacity=1 << 21, queue_capacity=n_requests),
        "served": gs.ServeConfig(max_views_per_batch=8, n_streams=1, pipeline_depth=2, slot_capacity=24_000_000,
                                 pair_capacity=96_000_000, pixel_capacity=1 << 24, queue_capacity=n_requests),
    }


def serve_oracle(gs, sc, offsets, table, trace, opts):
    """The FP64 oracle on sampled requests of the trace (the first of each
    resolution): the level-of-detail selection the server makes, then the
    oracle's projection, binning and compositing of exactly the selected
    Gaussians, on the host's threads; oracle req/s = requests / seconds."""
    import oracle
    picked, seen = [], set()
    for r in trace:
        key = (r["camera"].width, r["camera"].height)
        if key not in seen:
            seen.add(key)
            picked.append(r)
    opt = dict(sh_degree=opts.sh_degree, dilation=opts.dilation, aa=opts.aa, bg=opts.bg)
    secs, n_sel = 0.0, 0
    for r in picked:
        lv, tot = gs.lod_select(table, r["camera"], r["budget"])
        idx = [np.arange(offsets[l - 1, p], offsets[l - 1, p] + table.counts[l - 1, p]) for p, l in enumerate(lv) if l > 0]
        sub = sc.subset(np.concatenate(idx) if idx else np.zeros(0, np.int64))
        n_sel += sub.n
        a = time.perf_counter()
        oracle.forward(sub, r["camera"], opt)
        secs += time.perf_counter() - a
    return {"value": round(len(picked) / secs, 4), "unit": "req/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{len(picked)} requests (one per resolution, {n_sel} Gaussians selected in all)"}


def serve_bench(gs, S, torch, fine, opts, n_requests, modes=None, loads=("", "_800", "_burst"), with_cpu=False):
    """Open-loop serving trace on the level-of-detail stand-in of the urban
    block: levels of 1M, 3M and 6M Gaussians resident in HBM, 30 m render-time
    partitions, thresholds (30, 60, inf) m; Poisson arrivals at 150 req/s,
    resolutions 640x360 / 1280x720 / 1920x1080 and budgets 1M / 3M / 6M
    drawn uniformly.  Each configuration of `modes` (default serve_modes)
    runs the trace as scheduled, with the arrival times compressed to 800
    req/s ("_800", where batches form), and with every request arriving at
    once ("_burst": the saturated throughput).  Latency = completion -
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
    modes = modes or serve_modes(gs, n_requests)
    fast = [r["t"] * 150.0 / 800.0 for r in trace]
    arrivals = {"": [r["t"] for r in trace], "_800": fast, "_burst": [0.0] * len(trace)}
    runs = [(name + load, cfg, arrivals[load]) for load in loads for name, cfg in modes.items()]
    res = {}
    for name, cfg, arr in runs:
        srv = gs.Server(params, table, opts, cfg)
        t0 = srv.now() + 0.5
        for r, o, ta in zip(trace, outs, arr):
            srv.submit(r["camera"], r["budget"], o, t0 + ta)
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
                     "split_batches": st["split_batches"], "rebinned_batches": st["rebinned_batches"],
                     "est_over_actual": round(st["est_over_actual"], 3),
                     "completed": st["completed"], "failed": st["failed"]}
        print(f"# {name}: {res[name]}", file=sys.stderr, flush=True)
    res["trace"] = (f"{len(trace)} requests, Poisson {len(trace) / trace[-1]['t']:.0f} req/s over "
                    f"{trace[-1]['t']:.1f} s, offered {sum(npx) / trace[-1]['t'] / 1e6:.0f} Mpix/s")
    if with_cpu:
        del params, flat, outs
        res["oracle"] = serve_oracle(gs, sc, offsets, table, trace, opts)
        print(f"# serving oracle: {res['oracle']}", file=sys.stderr, flush=True)
    return res


def _ev(torch):
    ev = torch.cuda.Event(enable_timing=True)
    ev.record()
    return ev


def cpu_baseline(scene, cams, crop: int, aa: bool = True, repeats: int = 1):
    """The FP64 oracle on a bounded sample of the same workload: every
    Gaussian is projected and back-projected for cameras that see a centred
    1/crop of each view (same pose and focal length, tile-aligned), and
    binning, compositing and its backward run on those crops.  The full
    step is extrapolated as projection + projection backward + crop x
    (binning + compositing + compositing backward); crop 1 is the whole
    step, timed `repeats` times (median)."""
    import oracle
    import synthetic as S
    opt = dict(sh_degree=3, aa=aa)
    runs = []
    for _ in range(repeats):
        t = {"project": 0.0, "bin": 0.0, "render": 0.0, "render_bwd": 0.0, "project_bwd": 0.0}
        px_sub = px_all = 0
        for cam in cams:
            cw = max(16, int(round(cam.width / math.sqrt(crop) / 16)) * 16) if crop > 1 else cam.width
            ch = max(16, int(round(cam.height / math.sqrt(crop) / 16)) * 16) if crop > 1 else cam.height
            x0 = ((cam.width - cw) // 2) // 16 * 16
            y0 = ((cam.height - ch) // 2) // 16 * 16
            sub = S.Camera(cam.fx, cam.fy, cam.cx - x0, cam.cy - y0, cam.viewmat, cw, ch)
            px_sub += cw * ch
            px_all += cam.width * cam.height
            a = time.perf_counter()
            proj = oracle.project(scene, sub, **opt)
            t["project"] += time.perf_counter() - a
            a = time.perf_counter()
            keys = oracle.depth_key(proj["depth"])
            bins = oracle.bin_pairs(proj["rect"], proj["tiles"], keys, np.zeros(scene.n, np.int32), [sub])
            t["bin"] += time.perf_counter() - a
            twod = oracle._twod([proj])
            a = time.perf_counter()
            img = oracle.render_view(sub, opt, 0, twod, bins["pair_slot"], bins["ranges"], guard_eps=None)
            t["render"] += time.perf_counter() - a
            g = (np.sign(img["rgb"]) / img["rgb"].size, np.zeros_like(img["depth"]), np.zeros_like(img["alpha"]))
            a = time.perf_counter()
            d2 = np.zeros((scene.n, 10))
            oracle.render_bwd_view(sub, opt, 0, twod, bins["pair_slot"], bins["ranges"], *g, d2, None)
            t["render_bwd"] += time.perf_counter() - a
            grads = {"means": np.zeros((3, scene.n)), "scales": np.zeros((3, scene.n)),
                     "quats": np.zeros((4, scene.n)), "opacities": np.zeros(scene.n), "sh": np.zeros((16, 3, scene.n))}
            a = time.perf_counter()
            oracle.project_bwd(scene, sub, opt, d2, grads)
            t["project_bwd"] += time.perf_counter() - a
            del proj, bins, twod, img, d2, grads
        frac = px_sub / px_all
        full = t["project"] + t["project_bwd"] + (t["bin"] + t["render"] + t["render_bwd"]) / frac
        runs.append((full, t, frac))
    runs.sort(key=lambda r: r[0])
    full, t, frac = runs[len(runs) // 2]
    what = ("the whole step" if crop == 1 else
            f"all {scene.n} Gaussians projected and back-projected (FP64) for centred crops of {frac:.3f} of the "
            f"pixels of each of the {len(cams)} view(s); binning, compositing and its backward on those crops, "
            f"scaled by 1/{frac:.3f}")
    return {"value": round(1.0 / full, 5), "unit": "iters/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": what + (f", median of {repeats}" if repeats > 1 else ""),
            "seconds": {k: round(v, 3) for k, v in t.items()}, "extrapolated_s_per_iter": round(full, 3)}


if __name__ == "__main__":
    main()
