"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (from the float32 arithmetic of each stage):
  projection: mean2d |d| <= 1e-4 px; conic, opacity', depth, rgb relative
      <= 2e-6 (FP64 arithmetic rounded once to FP32);
  tile rectangles: inside the oracle's 3-sigma rectangles, empty where those
      are (Gaussians whose extent or mean sits within 1e-9 of an integer
      aside); tile culling: every (tile, Gaussian) pair where the oracle's
      FP64 record passes the skip rule at some pixel centre is listed, every
      listed pair lies in a 3-sigma rectangle, and the listed pairs beyond
      the needed ones stay below 10 %;
  binning and sort: bit-exact on the GPU's own records (stage-chained);
  compositing: max |d| <= 1e-4 on rgb and alpha, depth <= 1e-4 max(1, depth),
      outside the guard band (pixels where a skip, clamp or stop decision
      lies within the float32 error bound of oracle.DEFAULT_GUARD); a pixel
      inside it must match one of the results its flagged decisions allow
      (gpu_util.check_image), at most 1e-4 of the pixels unresolved;
  gradients: per group ||g - g_ref|| / ||g_ref|| <= 1e-3, and elementwise
      |g - g_ref| <= 1e-3 |g_ref| + 1e-3 rms(g_ref) for >= 99.9% of entries.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import synthetic as S
from gpu_util import (border_slots, check_image, check_tile_culling, decode_records, decode_rect, gpu_forward, grads_oracle_layout,
                      oracle_opt, to_dev, view_images)

pytestmark = pytest.mark.gpu


def small_cam(W, H, f, tz=4.0):
    vm = np.eye(4, dtype=np.float32)
    vm[2, 3] = tz
    return S.Camera(f, f, W / 2.0, H / 2.0, vm, W, H)


def oblique_cam(W, H, f):
    return S.Camera(f, f, W / 2.0, H / 2.0, S.look_at((1.6, -1.1, -3.3), (0.05, 0.1, 0.0), up=(0.3, -1, 0.2)), W, H)


def ring_cam(k, n=12):
    """One of n narrow views around the unit box from different directions,
    so that Gaussians are seen by many different subsets of the views."""
    a = 0.9 * np.pi * k / n
    sizes = ((48, 40), (64, 48), (37, 29), (80, 60))
    W, H = sizes[k % len(sizes)]
    eye = (3.5 * np.sin(a), 0.6 * np.sin(3 * a), -3.5 * np.cos(a))
    target = (0.4 * np.sin(2 * a), 0.3 * np.cos(3 * a), 0.0)
    return S.Camera(4.0 * W, 4.0 * W, W / 2.0, H / 2.0, S.look_at(eye, target, up=(0.0, -1.0, 0.0)), W, H)


CASES = {
    # name: (scene factory, cams, options)
    "c1": (lambda: S.scene_c1(), [S.camera_c1()], dict(aa=False)),
    "ragged_aa": (lambda: S.random_scene(3001, seed=5, log_scale_mu=-2.6), [oblique_cam(173, 91, 120.0)],
                  dict(aa=True, bg=(0.1, 0.2, 0.3))),
    "multiview": (lambda: S.random_scene(2500, seed=6, log_scale_mu=-2.5),
                  [S.camera_c1(), oblique_cam(100, 70, 80.0), small_cam(37, 53, 40.0)], dict(aa=True, sh_degree=2)),
    # twelve views: view masks beyond the low 8 bits, many distinct view sets per workgroup
    "manyview": (lambda: S.random_scene(1800, seed=8, log_scale_mu=-2.6), [ring_cam(k) for k in range(12)],
                 dict(aa=True)),
}


def _opts(gs, d):
    return gs.RenderOptions(**d)


@pytest.mark.parametrize("case", list(CASES))
def test_projection_matches_oracle(gpu_lib, case):
    make, cams, od = CASES[case]
    scene = make()
    opts = _opts(gpu_lib, od)
    params = to_dev(scene)
    proj = gpu_lib.project(*params, cams, opts)
    torch.cuda.synchronize()
    rec = proj.rec.cpu().numpy()
    tiles = proj.tiles.cpu().numpy()
    mask = proj.tile_mask.cpu().numpy().view(np.uint64)
    rect = decode_rect(proj.rect.cpu().numpy(), tiles, cams, scene.n, mask=mask)
    n = scene.n
    for v, c in enumerate(cams):
        p = oracle.project(scene, c, **oracle_opt(opts))
        sl = slice(v * n, (v + 1) * n)
        ok = ~border_slots([p])
        # the GPU rectangle is the oracle's 3-sigma rectangle narrowed by tile
        # culling (whose tiles are checked against the oracle's definition in
        # the binning tests): inside it, and empty where it is empty
        gt, pt = tiles[sl].astype(np.int64), p["tiles"].astype(np.int64)
        assert np.all(gt[ok] <= pt[ok]) and np.all(gt[ok & (pt == 0)] == 0)
        vis = (gt > 0) & ok
        r, q = rect[sl][vis], p["rect"][vis]
        assert np.all(r[:, :2] >= q[:, :2]) and np.all(r[:, 2:] <= q[:, 2:])
        assert vis.sum() > 10
        m2, con, op, rgb, dep = decode_records(rec[sl])
        np.testing.assert_allclose(m2[vis], p["mean2d"][vis], atol=1e-4, rtol=0)
        np.testing.assert_allclose(con[vis], p["conic"][vis], rtol=2e-6, atol=1e-7 * np.abs(p["conic"][vis]).max())
        np.testing.assert_allclose(op[vis], p["opac"][vis], rtol=2e-6, atol=1e-7)
        np.testing.assert_allclose(dep[vis], p["depth"][vis], rtol=2e-7)
        np.testing.assert_allclose(rgb[vis], p["rgb"][vis], rtol=2e-6, atol=2e-6)
        keys = proj.depth_key.cpu().numpy().view(np.uint32)[sl]
        np.testing.assert_array_equal(keys[vis], oracle.depth_key(p["depth"])[vis])
        assert np.all(keys[tiles[sl] == 0] == 0xFFFFFFFF)


@pytest.mark.parametrize("case", list(CASES))
def test_binning_bit_exact_stage_chained(gpu_lib, case):
    make, cams, od = CASES[case]
    scene = make()
    opts = _opts(gpu_lib, od)
    params, proj, pairs, ranges, P, _ = gpu_forward(gpu_lib, scene, cams, opts)
    tiles = proj.tiles.cpu().numpy()
    mask = proj.tile_mask.cpu().numpy().view(np.uint64)
    rect = decode_rect(proj.rect.cpu().numpy(), tiles, cams, scene.n, mask=mask)
    keys = proj.depth_key.cpu().numpy().view(np.uint32)
    slot_view = np.repeat(np.arange(len(cams), dtype=np.int32), scene.n)
    ref = oracle.bin_pairs(rect, tiles, keys, slot_view, cams, mask=mask)
    assert P == ref["n_pairs"] and P > 0
    np.testing.assert_array_equal(pairs.cpu().numpy().view(np.uint32), ref["pair_slot"])
    np.testing.assert_array_equal(ranges.cpu().numpy().view(np.uint32), ref["ranges"])
    # the GPU's culled tiles against the oracle's per-pixel definition
    f = oracle.forward(scene, cams, oracle_opt(opts), guard_eps=None)
    need, got, extra = check_tile_culling(f, pairs, ranges, P)
    print(f"{case}: {f['bins']['n_pairs']} pairs in 3-sigma rectangles, {need} needed, GPU {got} (+{extra})")
    assert extra <= 0.1 * need


@pytest.mark.parametrize("case", list(CASES))
def test_compositing_stage_chained(gpu_lib, case):
    """Oracle compositing in FP64 on the GPU's own records and pair lists."""
    make, cams, od = CASES[case]
    scene = make()
    opts = _opts(gpu_lib, od)
    params, proj, pairs, ranges, P, out = gpu_forward(gpu_lib, scene, cams, opts)
    twod = decode_records(proj.rec.cpu().numpy())
    pv = pairs.cpu().numpy().view(np.uint32)
    rg = ranges.cpu().numpy().view(np.uint32)
    toff = np.cumsum([0] + [c.n_tiles for c in cams])[:-1]
    gimgs = {k: view_images(out[k].cpu().numpy(), cams) for k in ("rgb", "depth", "alpha", "T", "last")}
    for v, c in enumerate(cams):
        ref = oracle.render_view(c, oracle_opt(opts), int(toff[v]), twod, pv, rg, guard_eps=oracle.STAGE_GUARD)
        g = {k: gimgs[k][v] for k in gimgs}
        check_image(c, oracle_opt(opts), int(toff[v]), twod, pv, rg, ref, g, f"{case} view {v} stage-chained",
                    guard_eps=oracle.STAGE_GUARD)
        same_last = (g["last"] == ref["last"]) | (ref["guard"] != 0)
        assert same_last.all()


@pytest.mark.parametrize("case", list(CASES))
def test_forward_end_to_end(gpu_lib, case):
    """GPU image from raw parameters vs the FP64 oracle from raw parameters."""
    make, cams, od = CASES[case]
    scene = make()
    opts = _opts(gpu_lib, od)
    _, _, _, _, P, out = gpu_forward(gpu_lib, scene, cams, opts)
    f = oracle.forward(scene, cams, oracle_opt(opts), guard_eps=oracle.DEFAULT_GUARD)
    assert f["bins"]["n_pairs"] >= P
    for v, c in enumerate(cams):
        g = {k: view_images(out[k].cpu().numpy(), cams)[v] for k in ("rgb", "depth", "alpha", "T", "last")}
        check_image(c, oracle_opt(opts), int(f["bins"]["tile_off"][v]), f["twod"], f["bins"]["pair_slot"],
                    f["bins"]["ranges"], f["images"][v], g, f"{case} view {v} end to end")


@pytest.mark.parametrize("case", ["c1", "ragged_aa"])
def test_alpha_box_covers_every_contribution(gpu_lib, case):
    """Each record's (hx, hy) box must contain every pixel centre where the
    entry's alpha o' G' reaches the skip threshold 1/255 (FP64 on the decoded
    record, with a relative slack of 1e-6 below the threshold); compositing
    leaves the entries outside the box unevaluated."""
    make, cams, od = CASES[case]
    scene = make()
    opts = _opts(gpu_lib, od)
    _, proj, pairs, ranges, P, _ = gpu_forward(gpu_lib, scene, cams, opts)
    rec = proj.rec.cpu().numpy()
    mean2d, conic, opac, _, _ = decode_records(rec)
    hx, hy = rec[:, 12].astype(np.float64), rec[:, 13].astype(np.float64)
    pv = pairs.cpu().numpy().view(np.uint32)[:P].astype(np.int64)
    rg = ranges.cpu().numpy().view(np.uint32).astype(np.int64)
    cam = cams[0]
    ys, xs = np.mgrid[0:16, 0:16]
    checked = 0
    for t in range(cam.n_tiles):
        sl = pv[rg[t, 0]:rg[t, 1]]
        if len(sl) == 0:
            continue
        px = (t % cam.tiles_x) * 16 + xs.ravel() + 0.5
        py = (t // cam.tiles_x) * 16 + ys.ravel() + 0.5
        inside = (px < cam.width) & (py < cam.height)
        dx = px[None, :] - mean2d[sl, 0:1]
        dy = py[None, :] - mean2d[sl, 1:2]
        A, B, C = conic[sl, 0:1], conic[sl, 1:2], conic[sl, 2:3]
        power = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy
        alpha = opac[sl, None] * np.exp(np.minimum(power, 0.0))
        hot = (alpha >= (1.0 - 1e-6) / 255.0) & (power <= 0) & inside[None, :]
        covered = (np.abs(dx) <= hx[sl, None]) & (np.abs(dy) <= hy[sl, None])
        assert np.all(covered[hot]), (t, int((hot & ~covered).sum()))
        checked += int(hot.sum())
    assert checked > 0


@pytest.mark.parametrize("case", ["c1", "multiview"])
def test_tile_order_is_a_longest_first_permutation(gpu_lib, case):
    make, cams, od = CASES[case]
    scene = make()
    _, proj, pairs, ranges, P, _ = gpu_forward(gpu_lib, scene, cams, _opts(gpu_lib, od))
    order = proj.tile_order.cpu().numpy().astype(np.int64)
    n_tiles = sum(c.n_tiles for c in cams)
    assert np.array_equal(np.sort(order), np.arange(n_tiles))
    rg = ranges.cpu().numpy().view(np.uint32).astype(np.int64)
    lens = (rg[:, 1] - rg[:, 0])[order]
    # non-increasing in 1/8-octave buckets of the list length
    assert np.all(np.diff(np.floor(8 * np.log2(lens + 1.0))) <= 0)


def test_render_count_is_consistent(gpu_lib):
    make, cams, od = CASES["ragged_aa"]
    scene = make()
    opts = _opts(gpu_lib, od)
    _, proj, pairs, ranges, P, out = gpu_forward(gpu_lib, scene, cams, opts)
    cnt = gpu_lib.render_count(proj, pairs, ranges, cams).cpu().numpy().astype(np.int64)
    last = out["last"].cpu().numpy().astype(np.int64)
    cam = cams[0]
    rg = ranges.cpu().numpy().view(np.uint32).astype(np.int64)
    py, px = np.divmod(np.arange(cam.n_pixels), cam.width)
    list_len = (rg[:, 1] - rg[:, 0])[(py // 16) * cam.tiles_x + px // 16]
    assert np.all(cnt[:, 1] <= cnt[:, 0]) and np.all(cnt[:, 0] <= list_len)
    assert np.all(cnt[:, 1] <= last)
    assert np.all(cnt[last > 0, 1] >= 1) and np.all(cnt[last == 0, 1] == 0)
    assert cnt[:, 1].sum() > 0


def _linear_loss_grads(gpu_lib, scene, cams, opts, seed=7):
    ws = [S.linear_loss_weights(c.height, c.width, seed=seed + v) for v, c in enumerate(cams)]
    params = to_dev(scene, requires_grad=True)
    stats = gpu_lib.RenderStats()
    rgb, depth, alpha = gpu_lib.rasterize(*params, cams, opts, stats)
    w_rgb = torch.from_numpy(np.concatenate([w[0].reshape(-1, 3) for w in ws])).cuda()
    w_d = torch.from_numpy(np.concatenate([w[1].reshape(-1) for w in ws])).cuda()
    w_a = torch.from_numpy(np.concatenate([w[2].reshape(-1) for w in ws])).cuda()
    loss = (w_rgb * rgb).sum() + (w_d * depth).sum() + (w_a * alpha).sum()
    loss.backward()
    torch.cuda.synchronize()
    return grads_oracle_layout(params), ws, stats


def _compare_grads(g, ref, groups=("means", "scales", "quats", "opacities", "sh")):
    for k in groups:
        a, b = g[k].ravel(), ref[k].ravel()
        nb = np.linalg.norm(b)
        assert nb > 0, k
        rel = np.linalg.norm(a - b) / nb
        assert rel <= 1e-3, (k, rel)
        rms = np.sqrt(np.mean(b * b))
        good = np.abs(a - b) <= 1e-3 * np.abs(b) + 1e-3 * rms
        assert good.mean() >= 0.999, (k, good.mean())


@pytest.mark.parametrize("case", list(CASES))
def test_gradients_match_oracle(gpu_lib, case):
    make, cams, od = CASES[case]
    scene = make()
    opts = _opts(gpu_lib, dict(od, absgrad=True))
    g, ws, stats = _linear_loss_grads(gpu_lib, scene, cams, opts)
    f = oracle.forward(scene, cams, oracle_opt(opts))
    ref = oracle.backward(scene, f, ws)
    _compare_grads(g, ref)
    norm = stats.mean2d_grad_norm.cpu().numpy()
    rn = ref["mean2d_norm"]
    assert np.linalg.norm(norm - rn) / np.linalg.norm(rn) <= 1e-3
    ab = stats.absgrad.cpu().numpy()
    assert np.linalg.norm(ab - ref["absgrad"]) / np.linalg.norm(ref["absgrad"]) <= 1e-3


def test_gradients_match_finite_differences(gpu_lib):
    """GPU gradient vs FP64 central differences of the oracle on 64 sampled
    parameters (8 per group, SH split into DC and higher bands)."""
    scene = S.random_scene(600, seed=12, log_scale_mu=-2.3)
    cam = oblique_cam(96, 72, 75.0)
    opts = gpu_lib.RenderOptions(aa=True, bg=(0.2, 0.3, 0.1))
    g, ws, _ = _linear_loss_grads(gpu_lib, scene, [cam], opts)
    w = ws[0]
    sc64 = S.Scene(*(np.asarray(a, np.float64).copy() for a in
                     (scene.means, scene.scales, scene.quats, scene.opacities, scene.sh)))
    od = oracle_opt(opts)

    def loss(sc):
        im = oracle.forward(sc, cam, od)["images"][0]
        return float((w[0] * im["rgb"]).sum() + (w[1] * im["depth"]).sum() + (w[2] * im["alpha"]).sum())

    def perturbed(group, idx, delta):
        arrs = {k: getattr(sc64, k).copy() for k in ("means", "scales", "quats", "opacities", "sh")}
        arrs[group][idx] += delta
        return S.Scene(arrs["means"], arrs["scales"], arrs["quats"], arrs["opacities"], arrs["sh"])

    f = oracle.forward(sc64, cam, od)
    vis = np.nonzero(f["proj"][0]["tiles"] > 0)[0]
    rng = np.random.default_rng(7)
    groups = [("means", (3,)), ("scales", (3,)), ("quats", (4,)), ("opacities", ()), ("sh_dc", (1, 3)),
              ("sh_rest", (15, 3)), ("means", (3,)), ("scales", (3,))]
    checked, total = 0, 0
    for gname, shape in groups:
        for _ in range(8):
            i = int(rng.choice(vis))
            if gname == "sh_dc":
                group, idx = "sh", (0, int(rng.integers(0, 3)), i)
            elif gname == "sh_rest":
                group, idx = "sh", (1 + int(rng.integers(0, 15)), int(rng.integers(0, 3)), i)
            else:
                group, idx = gname, tuple(int(rng.integers(0, s)) for s in shape) + (i,)
            theta = getattr(sc64, group)[idx]
            h = 1e-6 * max(1.0, abs(theta))
            fd = [(loss(perturbed(group, idx, k * h)) - loss(perturbed(group, idx, -k * h))) / (2 * k * h)
                  for k in (1, 2)]
            total += 1
            if abs(fd[0] - fd[1]) > 1e-4 * (abs(fd[0]) + 1e-6):
                continue      # a discrete event within 2h of theta
            rms = np.sqrt(np.mean(g[group] ** 2))
            assert abs(g[group][idx] - fd[0]) <= 1e-3 * abs(fd[0]) + 1e-3 * rms, (group, idx, g[group][idx], fd)
            checked += 1
    assert total == 64 and checked >= 56


def test_forward_is_deterministic(gpu_lib):
    scene = S.random_scene(5000, seed=9, log_scale_mu=-2.7)
    cams = [oblique_cam(200, 150, 150.0)]
    opts = gpu_lib.RenderOptions(aa=True)
    a = gpu_forward(gpu_lib, scene, cams, opts)[-1]
    b = gpu_forward(gpu_lib, scene, cams, opts)[-1]
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_backward_run_to_run_spread(gpu_lib):
    """The forward is atomic-free and bitwise repeatable; the backward sums
    per-pixel contributions with float atomics, whose order varies from run
    to run.  Over repeated runs on the same inputs each gradient group must
    stay within 1e-6 of its norm (relative spread, measured and printed)."""
    scene = S.random_scene(20000, seed=12, log_scale_mu=-3.0)
    cams = [oblique_cam(320, 240, 240.0), oblique_cam(160, 120, 120.0)]
    opts = gpu_lib.RenderOptions(aa=True, absgrad=True)
    params = to_dev(scene, requires_grad=True)
    gen = torch.Generator(device="cuda").manual_seed(4)
    npx = sum(c.width * c.height for c in cams)
    w = [torch.randn(sh, device="cuda", generator=gen) for sh in ((npx, 3), (npx,), (npx,))]
    runs, outs = [], []
    for _ in range(6):
        for p in params:
            p.grad = None
        stats = gpu_lib.RenderStats()
        rgb, depth, alpha = gpu_lib.rasterize(*params, cams, opts, stats)
        ((rgb * w[0]).sum() + (depth * w[1]).sum() + (alpha * w[2]).sum()).backward()
        runs.append([p.grad.detach().clone() for p in params] + [stats.mean2d_grad_norm.clone(),
                                                                   stats.absgrad.clone()])
        outs.append((rgb.detach().clone(), depth.detach().clone(), alpha.detach().clone()))
    for o in outs[1:]:
        assert all(torch.equal(a, b) for a, b in zip(outs[0], o))
    names = ("means", "scales", "quats", "opacities", "sh", "mean2d_grad_norm", "absgrad")
    spread = {}
    for k, name in enumerate(names):
        ref = runs[0][k].double()
        spread[name] = max(float((r[k].double() - ref).norm() / ref.norm()) for r in runs[1:])
    print("backward run-to-run relative spread:", {k: f"{v:.1e}" for k, v in spread.items()})
    assert max(spread.values()) < 1e-6, spread


def test_projection_backward_with_and_without_zeroed_outputs(gpu_lib):
    """gs_project_bwd writing every row (zeros for Gaussians no view sees)
    and, after gs_grads_zero, only the seen rows give the same gradients bit
    for bit; the first overwrites outputs that held NaN."""
    import ctypes as C
    from paper_2507_23006_amd import _lib as L
    from paper_2507_23006_amd.rasterizer import gaussians_struct
    scene = S.random_scene(30000, seed=14, log_scale_mu=-3.0)
    cams = [oblique_cam(160, 120, 400.0), oblique_cam(96, 80, 300.0)]     # narrow: about a quarter unseen
    opts = gpu_lib.RenderOptions(aa=True)
    params = to_dev(scene)
    proj = gpu_lib.project(*params, cams, opts)
    pairs, ranges, P = gpu_lib.bin_sort(proj, cams, scene.n)
    out = gpu_lib.render_fwd(proj, pairs, ranges, cams, opts)
    npx = sum(c.width * c.height for c in cams)
    gen = torch.Generator(device="cuda").manual_seed(8)
    d = [torch.randn(sh, device="cuda", generator=gen) for sh in ((npx, 3), (npx,), (npx,))]
    R = gpu_lib.rasterizer
    keep = R.FILL_BESIDE_MIN
    R.FILL_BESIDE_MIN = 0       # the second-stream fill at any size
    try:
        ref = gpu_lib.render_bwd(params, cams, opts, proj, pairs, ranges, out["T"], out["last"], *d)
    finally:
        R.FILL_BESIDE_MIN = keep
    torch.cuda.synchronize()
    seen = (proj.tiles.view(len(cams), -1) > 0).any(0)
    assert 0 < int(seen.sum()) < scene.n
    lib = L.load()
    grads = {k: torch.full_like(ref[k], float("nan")) for k in ("means", "scales", "quats", "opacities", "sh")}
    go = L.GsGaussiansGrad()
    go.d_means, go.d_scales, go.d_quats = grads["means"].data_ptr(), grads["scales"].data_ptr(), grads["quats"].data_ptr()
    go.d_opacities, go.d_sh = grads["opacities"].data_ptr(), grads["sh"].data_ptr()
    norm = torch.empty((len(cams), scene.n), device="cuda")
    g2 = gpu_lib.grad2d_view(ref)
    L.check(lib.gs_project_bwd(C.byref(gaussians_struct(*params)), L.make_cameras(cams), len(cams),
                               C.byref(opts.c()), C.byref(proj.c()), C.c_void_p(g2.data_ptr()), C.byref(go),
                               C.c_void_p(norm.data_ptr()), None, 0,
                               C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    torch.cuda.synchronize()
    for k, t in grads.items():
        assert torch.equal(t, ref[k]), k
    assert torch.equal(norm, ref["mean2d_grad_norm"])


def test_permutation_invariance_bitwise(gpu_lib):
    scene = S.random_scene(3000, seed=10, log_scale_mu=-2.7)
    cams = [oblique_cam(128, 96, 100.0)]
    # keep Gaussians whose float32 depth keys are distinct, so that the
    # depth order (and hence the image) does not depend on input order
    keys = oracle.depth_key(oracle.project(scene, cams[0])["depth"])
    _, first, counts = np.unique(keys, return_index=True, return_counts=True)
    scene = scene.subset(np.sort(first[counts == 1]))
    opts = gpu_lib.RenderOptions()
    a = gpu_forward(gpu_lib, scene, cams, opts)[-1]
    perm = np.random.default_rng(2).permutation(scene.n)
    b = gpu_forward(gpu_lib, scene.subset(perm), cams, opts)[-1]
    for k in ("rgb", "depth", "alpha", "T"):
        assert torch.equal(a[k], b[k]), k


def test_everything_culled(gpu_lib):
    scene = S.random_scene(1000, seed=3)
    cam = small_cam(64, 48, 50.0, tz=-10.0)      # all Gaussians behind the camera
    opts = gpu_lib.RenderOptions(bg=(0.5, 0.25, 1.0))
    _, proj, pairs, ranges, P, out = gpu_forward(gpu_lib, scene, [cam], opts)
    assert P == 0
    assert torch.all(out["T"] == 1.0) and torch.all(out["last"] == 0)
    assert torch.allclose(out["rgb"], torch.tensor([0.5, 0.25, 1.0], device="cuda").expand_as(out["rgb"]))
    params = to_dev(scene, requires_grad=True)
    rgb, depth, alpha = gpu_lib.rasterize(*params, [cam], opts)
    (rgb.sum() + depth.sum() + alpha.sum()).backward()
    for p in params:
        assert torch.all(p.grad == 0)


def test_single_gaussian_and_tiny_image(gpu_lib):
    sh = np.zeros((16, 3, 1), np.float32)
    sh[0, :, 0] = 1.0
    scene = S.Scene(np.array([[0.0], [0.0], [0.0]], np.float32), np.full((3, 1), 0.3, np.float32),
                    np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), np.array([0.7], np.float32), sh)
    for W, H in ((1, 1), (17, 3), (16, 16)):
        cam = small_cam(W, H, 20.0)
        opts = gpu_lib.RenderOptions(sh_degree=0)
        _, _, _, _, P, out = gpu_forward(gpu_lib, scene, [cam], opts)
        f = oracle.forward(scene, cam, oracle_opt(opts))
        ref = f["images"][0]
        assert 0 < P <= f["bins"]["n_pairs"]
        np.testing.assert_allclose(out["rgb"].cpu().numpy().reshape(H, W, 3), ref["rgb"], atol=1e-5)


def test_invalid_arguments_raise(gpu_lib):
    scene = S.random_scene(10, seed=1)
    params = to_dev(scene)
    opts = gpu_lib.RenderOptions()
    bad = small_cam(0, 10, 10.0)
    with pytest.raises(gpu_lib.GsError):
        gpu_lib.project(*params, [bad], opts)
    with pytest.raises(gpu_lib.GsError):
        gpu_lib.project(*params, [small_cam(10, 10, 10.0)] * 17, opts)
    with pytest.raises(gpu_lib.GsError):
        gpu_lib.project(*params, [small_cam(10, 10, 10.0)], gpu_lib.RenderOptions(sh_degree=4))


@pytest.mark.parametrize("n_pix,with_depth", [(1, True), (160 * 120, True), (1920 * 1080, True), (5000, False)])
def test_loss_kernel_matches_oracle(gpu_lib, n_pix, with_depth):
    from oracle import loss as OL
    rng = np.random.default_rng(n_pix)
    rgb, t_rgb = rng.random((n_pix, 3)).astype(np.float32), rng.random((n_pix, 3)).astype(np.float32)
    D = rng.uniform(0, 40, n_pix).astype(np.float32)
    a = rng.uniform(0, 1, n_pix).astype(np.float32)
    a[::97] = 0.0                                    # below the clamp
    td = rng.uniform(20, 45, n_pix).astype(np.float32) if with_depth else None
    dev = [torch.from_numpy(x).cuda().requires_grad_(True) for x in (rgb, D, a)]
    tt = [torch.from_numpy(t_rgb).cuda(), torch.from_numpy(td).cuda() if with_depth else None]
    loss = gpu_lib.l1_depth_loss(dev[0], dev[1], dev[2], tt[0], tt[1], 0.5)
    (2.0 * loss).backward()
    L, dr, dd, da = OL.l1_depth(rgb, D, a, t_rgb, td, 0.5)
    assert abs(loss.item() - L) <= 1e-6 * abs(L)
    np.testing.assert_allclose(dev[0].grad.cpu().numpy(), 2 * dr, rtol=1e-6, atol=0)
    np.testing.assert_allclose(dev[1].grad.cpu().numpy(), 2 * dd, rtol=2e-6, atol=0)
    np.testing.assert_allclose(dev[2].grad.cpu().numpy(), 2 * da, rtol=4e-6, atol=0)
    # the loss is summed in a fixed order
    again = gpu_lib.l1_depth_loss(dev[0], dev[1], dev[2], tt[0], tt[1], 0.5)
    assert torch.equal(loss, again)


def test_segmented_backward_matches_whole_lists(gpu_lib):
    """Lists longer than 512 positions are walked in segments by separate
    workgroups (state behind each segment folded from a pre-pass); the 2D
    gradients must equal those of whole-list walks to float rounding.  The
    walk without the AbsGS sums (a 10-field reduction) gives the same
    fields 0-9 and leaves fields 10 and 11 zero.  The segmented forward
    (gs_render_fwd_seg: long lists walked in segments by separate
    workgroups, folded, and the stop segment re-walked) agrees with the
    sequential walk to float rounding -- a stop decision may differ only
    where T is within rounding of the threshold -- and the backward that
    reads its segment states (seg_ready = 1) gives the gradients of the
    pre-pass over its own T_final and last."""
    import ctypes as C
    from paper_2507_23006_amd import _lib as L
    cam = S.Camera(60.0, 60.0, 24.0, 20.0, S.look_at((0.3, -0.2, -3.0), (0.0, 0.0, 0.0)), 48, 40)
    scene = S.random_scene(6000, seed=3, log_scale_mu=-3.2)
    opts = gpu_lib.RenderOptions(aa=True, bg=(0.1, 0.2, 0.3))
    _, proj, pairs, ranges, P, _ = gpu_forward(gpu_lib, scene, [cam], opts)
    out = gpu_lib.render_fwd(proj, pairs, ranges, [cam], opts, seg=False)     # every list walked whole
    rg = ranges.cpu().numpy().view(np.uint32).astype(np.int64)
    assert (rg[:, 1] - rg[:, 0]).max() > 1024          # several segments per long list
    lib = L.load()
    n_slots, npx = scene.n, cam.n_pixels
    gen = torch.Generator(device="cuda").manual_seed(1)
    d = [torch.randn(s, device="cuda", generator=gen) for s in ((npx, 3), (npx,), (npx,))]
    # the segmented forward against the sequential one
    fseg = gpu_lib.seg_workspace([cam], pairs)
    out2 = gpu_lib.render_fwd(proj, pairs, ranges, [cam], opts, seg=fseg)
    torch.cuda.synchronize()
    # a stop decision may differ only where T is within rounding of the
    # threshold: then last differs and the colour by at most that entry's
    moved = out["last"].cpu().numpy() != out2["last"].cpu().numpy()
    print(f"segmented forward: {int(moved.sum())} of {moved.size} pixels stop elsewhere")
    assert moved.mean() <= 1e-3
    T1, T2 = out["T"].cpu().numpy(), out2["T"].cpu().numpy()
    assert np.all(np.minimum(T1, T2)[moved] < 1e-3)
    for k, tol in (("rgb", 2e-5), ("depth", 2e-5), ("alpha", 2e-5), ("T", 2e-5)):
        a1, a2 = out[k].cpu().numpy().reshape(len(moved), -1), out2[k].cpu().numpy().reshape(len(moved), -1)
        scale = max(1.0, float(np.abs(a1).max()))
        assert np.abs(a1 - a2)[~moved].max() <= tol * scale, k
        if moved.any():
            assert np.abs(a1 - a2)[moved].max() <= 1e-3 * scale, k
    # an area with room for one segment state: the plan keeps every list
    # whole, and the images are those of the plain forward bit for bit
    small = torch.empty(lib.gs_seg_workspace_size(cam.n_tiles, 0) + 256, dtype=torch.uint8, device="cuda")
    out3 = gpu_lib.render_fwd(proj, pairs, ranges, [cam], opts, seg=small)
    torch.cuda.synchronize()
    for k in ("rgb", "depth", "alpha", "T", "last"):
        assert torch.equal(out[k], out3[k]), k
    res = []
    # (segmented, AbsGS sums, states from the segmented forward, forward used)
    runs = ((False, 1, 0, out), (True, 1, 0, out), (True, 0, 0, out), (True, 1, 1, out2), (True, 1, 0, out2))
    for seg, absum, ready, fo in runs:
        g2 = torch.zeros((n_slots, 12), device="cuda")
        if ready:
            base = (fseg.data_ptr() + 255) & ~255
            sp, ssz = C.c_void_p(base), fseg.numel() - (base - fseg.data_ptr())
        else:
            ssz = lib.gs_seg_workspace_size(cam.n_tiles, P) if seg else 0
            sbuf = torch.empty(ssz + 512, dtype=torch.uint8, device="cuda")
            sp = C.c_void_p((sbuf.data_ptr() + 255) & ~255) if seg else None
        L.check(lib.gs_composite_bwd(C.byref(proj.c()), C.c_void_p(pairs.data_ptr()), C.c_void_p(ranges.data_ptr()),
                                     L.make_cameras([cam]), 1, C.byref(opts.c()), C.c_void_p(fo["T"].data_ptr()),
                                     C.c_void_p(fo["last"].data_ptr()), *[C.c_void_p(t.data_ptr()) for t in d],
                                     absum, n_slots, C.c_void_p(g2.data_ptr()), sp, ssz, ready,
                                     C.c_void_p(torch.cuda.current_stream().cuda_stream)))
        torch.cuda.synchronize()
        res.append(g2.cpu().numpy().astype(np.float64) * (proj.tiles.cpu().numpy()[:, None] > 0))
    a, b, c, e, f = res
    rel = np.linalg.norm(e - f, axis=0) / np.maximum(np.linalg.norm(f, axis=0), 1e-30)
    assert rel.max() < 1e-5, rel
    rel = np.linalg.norm(a - b, axis=0) / np.maximum(np.linalg.norm(a, axis=0), 1e-30)
    assert rel.max() < 1e-5, rel
    assert np.linalg.norm(a[:, 10:], axis=0).min() > 0
    assert not c[:, 10:].any()
    rel = np.linalg.norm(c[:, :10] - b[:, :10], axis=0) / np.maximum(np.linalg.norm(b[:, :10], axis=0), 1e-30)
    assert rel.max() < 1e-5, rel


@pytest.mark.parametrize("W,H", [(1, 1), (16, 16), (37, 23), (1920, 1080)])
def test_dssim_kernel_matches_oracle(gpu_lib, W, H):
    from oracle import ssim as OS
    rng = np.random.default_rng(W * 7 + H)
    x = rng.random((H, W, 3)).astype(np.float32)
    y = np.clip(x + 0.1 * rng.standard_normal((H, W, 3)), 0, 1).astype(np.float32)
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    loss = gpu_lib.dssim_loss(xt, torch.from_numpy(y).cuda(), 0.2)
    (3.0 * loss).backward()
    L, g = OS.dssim(x, y, 0.2)
    assert abs(loss.item() - L) <= 1e-5 * max(abs(L), 1e-3)
    got = xt.grad.cpu().numpy().astype(np.float64)
    scale = np.abs(3 * g).max()
    assert np.abs(got - 3 * g).max() <= 1e-4 * scale
    again = gpu_lib.dssim_loss(xt, torch.from_numpy(y).cuda(), 0.2)
    assert torch.equal(loss, again)


def test_async_binning_matches_and_reports_overflow(gpu_lib):
    """gs_bin_sort reads nothing back: with sync=False the pair count stays
    on the device (PairCount), results equal the synchronous call's bit for
    bit, a pair buffer that is too small shows in the count and leaves every
    tile list empty, and the autograd path raises at the end of the backward
    when its forward's binning overflowed (after growing the capacity)."""
    make, cams, od = CASES["multiview"]
    scene = make()
    opts = _opts(gpu_lib, od)
    params = to_dev(scene)
    proj = gpu_lib.project(*params, cams, opts)
    pv, rg, P = gpu_lib.bin_sort(proj, cams, scene.n)
    pv2, rg2, P2 = gpu_lib.bin_sort(proj, cams, scene.n, sync=False, capacity_hint=P + 10)
    assert int(P2) == P and not P2.overflowed()
    assert torch.equal(pv2[:P], pv) and torch.equal(rg2, rg)
    pv3, rg3, P3 = gpu_lib.bin_sort(proj, cams, scene.n, sync=False, capacity_hint=P // 2)
    assert int(P3) == P and P3.overflowed()
    assert int(rg3.to(torch.int64).abs().sum()) == 0
    # more asynchronous counts in flight than the pinned slots they are read
    # through, two different counts alternating, read only at the end
    half = gpu_lib.project(*params, cams[:1], opts)
    P_half = int(gpu_lib.bin_sort(half, cams[:1], scene.n)[2])
    assert P_half != P
    n_ring = gpu_lib.rasterizer._PinnedRing.SLOTS
    counts = [gpu_lib.bin_sort(*((proj, cams) if i % 2 == 0 else (half, cams[:1])), scene.n, sync=False,
                               capacity_hint=P + 10)[2] for i in range(n_ring + 40)]
    assert [int(c) for c in counts] == [P if i % 2 == 0 else P_half for i in range(len(counts))]
    ws = gpu_lib.rasterizer._default_ws
    key = (scene.n * len(cams), sum(c.n_tiles for c in cams))
    saved = ws.pair_caps.get(key)
    ws.pair_caps[key] = P // 2
    try:
        prm = to_dev(scene, requires_grad=True)
        rgb, depth, alpha = gpu_lib.rasterize(*prm, cams, opts)
        with pytest.raises(gpu_lib.GsError):
            rgb.sum().backward()
        assert ws.pair_caps[key] > P
    finally:
        if saved is None:
            ws.pair_caps.pop(key, None)
        else:
            ws.pair_caps[key] = saved
