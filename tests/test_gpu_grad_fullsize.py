"""Gradient parity at the full sizes of the benchmark configurations.

The loss is a random linear functional of the rendered rgb, accumulated
depth and alpha (weights N(0, 1), seed 7): it has no kinks, so its upstream
gradient is exact and the comparison tests the rasterizer's backward alone.

* C3 (6M-Gaussian urban block, 1920x1080, anti-aliasing): every parameter
  group over all Gaussians against the FP64 oracle's analytic gradient, the
  per-view |dL/d mean2d| and the AbsGS accumulation; and 64 sampled
  parameters (8 per group, SH split into DC and higher bands) against FP64
  central differences, re-rendering only the tiles of the perturbed
  Gaussian's rectangle (the rest of the image cannot change) and drawing a
  new sample whenever the perturbation changes the discrete signature (the
  rectangle, the depth order in those tiles, the last composited positions)
  or the two step sizes disagree.
* C2 (1M Gaussians, 1600x1066): every group, and |dL/d mean2d}.
* C5 (12M Gaussians, eight views of mixed resolution, one multi-view
  launch with gradients accumulated across views): the loss is supported on
  sampled tiles of every view (each view's longest list and two random
  ones), so the oracle can compute it from those tiles alone -- per view,
  from its own FP64 projection of the Gaussians the tiles list -- and the
  GPU's accumulated gradient must equal the sum over views on those
  Gaussians and vanish on all others; two views are also compared alone.
"""
import numpy as np
import pytest
import torch

import oracle
import synthetic as S
from gpu_util import compare_grad, gpu_forward, grads_oracle_layout, linear_loss, oracle_opt, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GROUPS = ("means", "scales", "quats", "opacities", "sh")


def _gpu_grads(gpu_lib, scene, cams, opts, ws):
    params = to_dev(scene, requires_grad=True)
    stats = gpu_lib.RenderStats()
    rgb, depth, alpha = gpu_lib.rasterize(*params, cams, opts, stats)
    linear_loss(ws, rgb, depth, alpha).backward()
    torch.cuda.synchronize()
    return params, stats


@pytest.fixture(scope="module")
def c3_grads(gpu_lib):
    scene, cam = S.scene_c3(seed=0), S.camera_c3(seed=2)
    opts = gpu_lib.RenderOptions(sh_degree=3, aa=True, absgrad=True)
    w = S.linear_loss_weights(cam.height, cam.width, seed=7)
    params, stats = _gpu_grads(gpu_lib, scene, [cam], opts, [w])
    g = grads_oracle_layout(params)
    del params
    f = oracle.forward(scene, cam, oracle_opt(opts), guard_eps=None)
    ref = oracle.backward(scene, f, [w])
    return dict(scene=scene, cam=cam, opts=opts, w=w, g=g, stats=stats, f=f, ref=ref)


def test_c3_gradients(c3_grads):
    g, ref, stats = c3_grads["g"], c3_grads["ref"], c3_grads["stats"]
    rels = {k: compare_grad(g[k], ref[k], k) for k in GROUPS}
    rels["mean2d_norm"] = compare_grad(stats.mean2d_grad_norm.cpu().numpy(), ref["mean2d_norm"], "mean2d_norm")
    rels["absgrad"] = compare_grad(stats.absgrad.cpu().numpy(), ref["absgrad"], "absgrad")
    print("C3 gradient relative errors: " + ", ".join(f"{k} {v:.1e}" for k, v in rels.items()))


def _tile_loss(cam, od, w, twod_loc, lists, tiles):
    """The linear loss over the given tiles, rendered from local records and
    lists; also the last composited positions there."""
    ps = np.concatenate(lists).astype(np.uint32)
    rg = np.zeros((cam.n_tiles, 2), np.uint32)
    mask = np.zeros(cam.n_tiles, np.uint8)
    off = 0
    for t, l in zip(tiles, lists):
        rg[t] = (off, off + len(l))
        mask[t] = 1
        off += len(l)
    im = oracle.render_view(cam, od, 0, twod_loc, ps, rg, tile_mask=mask, guard_eps=None)
    loss = float((w[0] * im["rgb"]).sum() + (w[1] * im["depth"]).sum() + (w[2] * im["alpha"]).sum())
    return loss, im["last"]


def test_c3_finite_differences(c3_grads):
    scene, cam, w, g, f, ref = (c3_grads[k] for k in ("scene", "cam", "w", "g", "f", "ref"))
    od = oracle_opt(c3_grads["opts"])
    p0 = f["proj"][0]
    keys = oracle.depth_key(p0["depth"])
    ps_all = f["bins"]["pair_slot"].astype(np.int64)
    rg_all = f["bins"]["ranges"].astype(np.int64)
    twod = f["twod"]
    # Gaussians that a pixel composited (a nonzero 2D gradient), with small rectangles
    contributed = np.any(ref["d2"] != 0.0, axis=1)
    small = (p0["tiles"] > 0) & (p0["tiles"] <= 64)
    pool = np.nonzero(contributed & small)[0]
    assert len(pool) > 10000
    rng = np.random.default_rng(7)
    groups = [("means", (3,)), ("scales", (3,)), ("quats", (4,)), ("opacities", ()), ("sh_dc", (1, 3)),
              ("sh_rest", (15, 3)), ("means", (3,)), ("scales", (3,))]
    rms = {k: float(np.sqrt(np.mean(g[k] ** 2))) for k in GROUPS}
    checked = redrawn = 0
    worst = 0.0
    for gname, shape in groups:
        done = 0
        while done < 8:
            assert redrawn < 200, "too many samples with a discrete event"
            i = int(rng.choice(pool))
            if gname == "sh_dc":
                group, idx = "sh", (0, int(rng.integers(0, 3)))
            elif gname == "sh_rest":
                group, idx = "sh", (1 + int(rng.integers(0, 15)), int(rng.integers(0, 3)))
            else:
                group, idx = gname, tuple(int(rng.integers(0, s)) for s in shape)
            x0, y0, x1, y1 = (int(v) for v in p0["rect"][i])
            tiles = [ty * cam.tiles_x + tx for ty in range(y0, y1 + 1) for tx in range(x0, x1 + 1)]
            lists = [ps_all[rg_all[t, 0]:rg_all[t, 1]] for t in tiles]
            uniq, inv = np.unique(np.concatenate(lists), return_inverse=True)
            loc_lists = np.split(inv, np.cumsum([len(l) for l in lists])[:-1])
            li = int(np.searchsorted(uniq, i))
            one = scene.subset(np.array([i]))
            arrs = {k: np.asarray(getattr(one, k), np.float64).copy() for k in GROUPS}
            theta = float(arrs[group][idx + (0,)])
            h = 1e-6 * max(1.0, abs(theta))

            def evaluate(delta):
                a = {k: v.copy() for k, v in arrs.items()}
                a[group][idx + (0,)] = theta + delta
                p = oracle.project(S.Scene(a["means"], a["scales"], a["quats"], a["opacities"], a["sh"]), cam, **od)
                if not p["visible"][0] or tuple(p["rect"][0]) != (x0, y0, x1, y1):
                    return None
                k_new = keys[uniq].copy()
                k_new[li] = oracle.depth_key(p["depth"])[0]
                for l in loc_lists:          # the depth order in every tile must stay
                    if not np.array_equal(np.lexsort((uniq[l], k_new[l])), np.arange(len(l))):
                        return None
                loc = [np.asarray(a_[uniq], np.float64).copy() for a_ in twod]
                for a_, k in zip(loc, ("mean2d", "conic", "opac", "rgb", "depth")):
                    a_[li] = p[k][0]
                return _tile_loss(cam, od, w, tuple(loc), loc_lists, tiles)

            ev = [evaluate(s * k * h) for k in (1, 2) for s in (1, -1)]
            if any(e is None for e in ev) or not all(np.array_equal(ev[0][1], e[1]) for e in ev[1:]):
                redrawn += 1
                continue
            fd = [(ev[0][0] - ev[1][0]) / (2 * h), (ev[2][0] - ev[3][0]) / (4 * h)]
            if abs(fd[0] - fd[1]) > 1e-4 * (abs(fd[0]) + 1e-6):
                redrawn += 1
                continue
            got = g[group][idx + (i,)]
            err = abs(got - fd[0])
            assert err <= 1e-3 * abs(fd[0]) + 1e-3 * rms[group], (gname, i, idx, got, fd)
            worst = max(worst, err / (abs(fd[0]) + rms[group]))
            done += 1
            checked += 1
    print(f"C3 FD: {checked} parameters checked, {redrawn} redrawn, worst |g - fd| / (|fd| + rms) {worst:.1e}")
    assert checked == 64


def test_c2_gradients(gpu_lib):
    scene, cam = S.scene_c2(seed=0), S.camera_c2()
    opts = gpu_lib.RenderOptions(sh_degree=3, aa=False)
    w = S.linear_loss_weights(cam.height, cam.width, seed=7)
    params, stats = _gpu_grads(gpu_lib, scene, [cam], opts, [w])
    g = grads_oracle_layout(params)
    f = oracle.forward(scene, cam, oracle_opt(opts), guard_eps=None)
    ref = oracle.backward(scene, f, [w], absgrad=False)
    rels = {k: compare_grad(g[k], ref[k], k) for k in GROUPS}
    rels["mean2d_norm"] = compare_grad(stats.mean2d_grad_norm.cpu().numpy(), ref["mean2d_norm"], "mean2d_norm")
    print("C2 gradient relative errors: " + ", ".join(f"{k} {v:.1e}" for k, v in rels.items()))


def _gather(params, idx):
    """Parameter gradients of the given Gaussians, in the oracle's layouts."""
    ii = torch.from_numpy(idx).cuda()
    out = {}
    for k, p in zip(GROUPS, params):
        gsel = p.grad.index_select(0, ii) if k == "sh" else p.grad.index_select(p.grad.dim() - 1, ii)
        a = gsel.cpu().numpy().astype(np.float64)
        out[k] = np.ascontiguousarray(a.transpose(1, 2, 0)) if k == "sh" else a
    return out


def test_c5_backward_sampled(gpu_lib):
    scene = S.scene_urban(12_000_000, 400, seed=0)
    cams = S.cameras_c5()
    n = scene.n
    opts = gpu_lib.RenderOptions(sh_degree=3, aa=True)
    od = oracle_opt(opts)
    _, _, pairs, ranges, P, _ = gpu_forward(gpu_lib, scene, cams, opts)
    rg = ranges.cpu().numpy().view(np.uint32).astype(np.int64)
    pv = pairs.cpu().numpy().view(np.uint32)[:P].astype(np.int64)
    del pairs, ranges
    toff = np.cumsum([0] + [c.n_tiles for c in cams])[:-1]
    rng = np.random.default_rng(11)
    # sampled tiles per view, and the loss weights supported on them
    picked, ws = [], []
    for v, cam in enumerate(cams):
        lens = rg[toff[v]:toff[v] + cam.n_tiles, 1] - rg[toff[v]:toff[v] + cam.n_tiles, 0]
        nonempty = np.nonzero(lens)[0]
        ts = sorted({int(np.argmax(lens))} | {int(t) for t in rng.choice(nonempty, 2, replace=False)})
        picked.append(ts)
        w = S.linear_loss_weights(cam.height, cam.width, seed=7 + v)
        keep = np.zeros((cam.height, cam.width), bool)
        for t in ts:
            keep[(t // cam.tiles_x) * 16:(t // cam.tiles_x + 1) * 16, (t % cam.tiles_x) * 16:(t % cam.tiles_x + 1) * 16] = True
        ws.append(tuple(np.where(keep[..., None] if a.ndim == 3 else keep, a, 0).astype(np.float32) for a in w))
    # oracle, per view: FP64 projection of the listed Gaussians, the sampled
    # tiles rendered and differentiated, chained to the parameters
    per_view = []
    for v, cam in enumerate(cams):
        lists = [pv[rg[toff[v] + t, 0]:rg[toff[v] + t, 1]] - v * n for t in picked[v]]
        gidx, inv = np.unique(np.concatenate(lists), return_inverse=True)
        sub = scene.subset(gidx)
        p = oracle.project(sub, cam, **od)
        assert np.all(p["visible"] == 1), v
        twod = (p["mean2d"], p["conic"], p["opac"], p["rgb"], p["depth"])
        ps = inv.astype(np.uint32)
        rgl = np.zeros((cam.n_tiles, 2), np.uint32)
        mask = np.zeros(cam.n_tiles, np.uint8)
        off = 0
        for t, l in zip(picked[v], lists):
            rgl[t] = (off, off + len(l))
            mask[t] = 1
            off += len(l)
        d2 = np.zeros((len(gidx), 10))
        oracle.render_bwd_view(cam, od, 0, twod, ps, rgl, *ws[v], d2, None, tile_mask=mask)
        gv = {"means": np.zeros((3, len(gidx))), "scales": np.zeros((3, len(gidx))),
              "quats": np.zeros((4, len(gidx))), "opacities": np.zeros(len(gidx)),
              "sh": np.zeros((16, 3, len(gidx)))}
        norm = oracle.project_bwd(sub, cam, od, d2, gv)
        per_view.append((gidx, gv, norm))
    union = np.unique(np.concatenate([pvw[0] for pvw in per_view]))
    total = {k: np.zeros(getattr(scene, k).shape[:-1] + (len(union),)) for k in GROUPS}
    for gidx, gv, _ in per_view:
        pos = np.searchsorted(union, gidx)
        for k in GROUPS:
            total[k][..., pos] += gv[k]
    # GPU: one multi-view launch, gradients accumulated across the views
    params, stats = _gpu_grads(gpu_lib, scene, cams, opts, ws)
    got = _gather(params, union)
    for k in GROUPS:
        compare_grad(got[k], total[k], f"C5 accumulated {k}")
    nz = torch.zeros(n, dtype=torch.bool, device="cuda")
    for k, p in zip(GROUPS, params):
        gg = p.grad.reshape(-1, n) if k != "sh" else p.grad.reshape(n, -1).t()
        nz |= (gg != 0).any(0)
    outside = np.setdiff1d(torch.nonzero(nz).flatten().cpu().numpy(), union)
    assert len(outside) == 0, f"{len(outside)} Gaussians outside the sampled tiles have a gradient"
    norms = stats.mean2d_grad_norm
    for v, (gidx, _, norm) in enumerate(per_view):
        compare_grad(norms[v].index_select(0, torch.from_numpy(gidx).cuda()).cpu().numpy(), norm,
                     f"C5 view {v} |dL/d mean2d|")
    del params, stats
    # two views alone (the others' weights zero)
    for v in (0, 6):
        wv = [ws[u] if u == v else tuple(np.zeros_like(a) for a in ws[u]) for u in range(len(cams))]
        params, _ = _gpu_grads(gpu_lib, scene, cams, opts, wv)
        gidx, gv, _ = per_view[v]
        got = _gather(params, gidx)
        for k in GROUPS:
            compare_grad(got[k], gv[k], f"C5 view {v} alone {k}")
        del params
    print(f"C5 backward: {len(union)} Gaussians in {sum(len(t) for t in picked)} sampled tiles of 8 views")
