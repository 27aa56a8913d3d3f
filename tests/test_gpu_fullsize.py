"""Parity at the full sizes of the benchmark configurations.

C3 (the benchmark: 6M-Gaussian urban block, 1920x1080, anti-aliasing, the
calls bench.py times) and C2 (1M Gaussians, 1600x1066): the FP64 oracle
renders the whole image (OpenMP over tiles, tens of seconds on the host), so
the comparison covers every pixel; C3 gradients are compared per parameter
group over all Gaussians.  C5 (12M Gaussians, eight views of 2x 3840x2160,
3x 1920x1080, 3x 1280x720 in one multi-view launch) is checked on samples
the oracle computes one by one: the projection of 40000 random Gaussians in
every view, the pair lists of the longest and a random tile of every view
rebuilt from the GPU's own rectangles and keys, and those tiles' pixels
composited by the oracle from the GPU's records."""
import numpy as np
import pytest
import torch

import oracle
import synthetic as S
from gpu_util import (border_slots, check_image, check_tile_culling, decode_records, decode_rect, gpu_forward, grads_oracle_layout,
                      mask_covers, mask_rows, oracle_opt, to_dev, view_images)

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def c3():
    return S.scene_c3(seed=0), S.camera_c3(seed=2)


def _forward_at_size(gpu_lib, scene, cams, opts, label):
    """Projection, binning and image of one full-size view against the FP64
    oracle: rectangles inside the oracle's 3-sigma rectangles, depth keys
    equal, binning bit-exact on the GPU's own rectangles, tile masks and keys
    (stage-chained), tile culling against the oracle's per-pixel definition,
    and the image against the unculled oracle (gpu_util.check_image)."""
    _, proj, pairs, ranges, P, out = gpu_forward(gpu_lib, scene, cams, opts)
    tiles = proj.tiles.cpu().numpy()
    mask = proj.tile_mask.cpu().numpy().view(np.uint64)
    rect = decode_rect(proj.rect.cpu().numpy(), tiles, cams, scene.n, mask=mask)
    keys = proj.depth_key.cpu().numpy().view(np.uint32)
    f = oracle.forward(scene, cams, oracle_opt(opts), guard_eps=oracle.DEFAULT_GUARD)
    p = f["proj"][0]
    ok = ~border_slots([p])
    gt, pt = tiles.astype(np.int64), p["tiles"].astype(np.int64)
    assert np.all(gt[ok] <= pt[ok]) and np.all(gt[ok & (pt == 0)] == 0)
    vis = gt > 0
    assert np.all(rect[vis & ok][:, :2] >= p["rect"][vis & ok][:, :2])
    assert np.all(rect[vis & ok][:, 2:] <= p["rect"][vis & ok][:, 2:])
    assert np.array_equal(keys[vis], oracle.depth_key(p["depth"])[vis])
    ref_bins = oracle.bin_pairs(rect, tiles, keys, np.zeros(scene.n, np.int32), cams, mask=mask)
    assert P == ref_bins["n_pairs"]
    assert np.array_equal(pairs.cpu().numpy().view(np.uint32)[:P], ref_bins["pair_slot"])
    assert np.array_equal(ranges.cpu().numpy().view(np.uint32), ref_bins["ranges"])
    need, got, extra = check_tile_culling(f, pairs, ranges, P)
    print(f"{label}: {f['bins']['n_pairs']} pairs in 3-sigma rectangles, {need} needed, GPU {got} (+{extra})")
    assert extra <= 0.1 * need
    g = {k: view_images(out[k].cpu().numpy(), cams)[0] for k in ("rgb", "depth", "alpha")}
    check_image(cams[0], oracle_opt(opts), 0, f["twod"], f["bins"]["pair_slot"], f["bins"]["ranges"],
                f["images"][0], g, label)


def test_c3_forward_and_binning(gpu_lib, c3):
    scene, cam = c3
    _forward_at_size(gpu_lib, scene, [cam], gpu_lib.RenderOptions(sh_degree=3, aa=True), "C3")


def test_c2_forward_and_binning(gpu_lib):
    scene, cam = S.scene_c2(seed=0), S.camera_c2()
    _forward_at_size(gpu_lib, scene, [cam], gpu_lib.RenderOptions(sh_degree=3, aa=False), "C2")


def test_c5_multiview_sampled(gpu_lib):
    scene = S.scene_urban(12_000_000, 400, seed=0)
    cams = S.cameras_c5()
    n = scene.n
    opts = gpu_lib.RenderOptions(sh_degree=3, aa=True)
    _, proj, pairs, ranges, P, out = gpu_forward(gpu_lib, scene, cams, opts)
    rng = np.random.default_rng(5)
    toff = np.cumsum([0] + [c.n_tiles for c in cams])[:-1]

    # projection of sampled Gaussians, every view
    idx = np.sort(rng.choice(n, 40_000, replace=False))
    sub = scene.subset(idx)
    for v, cam in enumerate(cams):
        p = oracle.project(sub, cam, **oracle_opt(opts))
        sl = torch.from_numpy(v * n + idx).cuda()
        t_gpu = proj.tiles[sl].cpu().numpy().astype(np.int64)
        ok = ~border_slots([p])
        assert np.all(t_gpu[ok] <= p["tiles"][ok]) and np.all(t_gpu[ok & (p["tiles"] == 0)] == 0), v
        vis = (t_gpu > 0) & ok
        assert vis.sum() > 100, v
        m2, con, op, rgb, dep = decode_records(proj.rec[sl].cpu().numpy())
        np.testing.assert_allclose(m2[vis], p["mean2d"][vis], atol=1e-4, rtol=0)
        np.testing.assert_allclose(con[vis], p["conic"][vis], rtol=2e-6, atol=1e-7 * np.abs(p["conic"][vis]).max())
        np.testing.assert_allclose(op[vis], p["opac"][vis], rtol=2e-6, atol=1e-7)
        np.testing.assert_allclose(dep[vis], p["depth"][vis], rtol=2e-7)
        np.testing.assert_allclose(rgb[vis], p["rgb"][vis], rtol=2e-6, atol=2e-6)

    # pair lists of sampled tiles, from the GPU's own rectangles and depth keys
    rg = ranges.cpu().numpy().view(np.uint32).astype(np.int64)
    pv = pairs.cpu().numpy().view(np.uint32)[:P]
    keys_all = proj.depth_key.cpu().numpy().view(np.uint32)
    tiles_all = proj.tiles.cpu().numpy().astype(np.int64)
    words = proj.rect.cpu().numpy().view(np.uint32).astype(np.int64)
    masks_all = proj.tile_mask.cpu().numpy().view(np.uint64)
    picked = []
    for v, cam in enumerate(cams):
        nt = cam.n_tiles
        lens = rg[toff[v]:toff[v] + nt, 1] - rg[toff[v]:toff[v] + nt, 0]
        nonempty = np.nonzero(lens)[0]
        sl = slice(v * n, (v + 1) * n)
        base, w, tl = words[sl, 0] - toff[v], words[sl, 1] & 0xFFFF, tiles_all[sl]
        seen = tl > 0
        x0 = np.where(seen, base % cam.tiles_x, 0)
        y0 = np.where(seen, base // cam.tiles_x, 0)
        mv = np.where(seen, masks_all[sl], np.uint64(0))
        h = np.where(seen, tl // np.maximum(w, 1), 0)
        h = np.where(mv != 0, mask_rows(mv, w), h)
        for t in (int(np.argmax(lens)), int(rng.choice(nonempty))):
            tx, ty = t % cam.tiles_x, t // cam.tiles_x
            cover = seen & (x0 <= tx) & (tx < x0 + w) & (y0 <= ty) & (ty < y0 + h)
            cover &= mask_covers(mv, w, x0, y0, tx, ty)
            slots = np.nonzero(cover)[0] + v * n
            want = slots[np.lexsort((slots, keys_all[slots]))].astype(np.uint32)
            got = pv[rg[toff[v] + t, 0]:rg[toff[v] + t, 1]]
            assert np.array_equal(got, want), (v, t)
            picked.append((v, t))

    # compositing of the sampled tiles by the oracle from the GPU's records
    imgs = {k: view_images(out[k].cpu().numpy(), cams) for k in ("rgb", "depth", "alpha")}
    for v, cam in enumerate(cams):
        ts = [t for (vv, t) in picked if vv == v]
        lists = [pv[rg[toff[v] + t, 0]:rg[toff[v] + t, 1]] for t in ts]
        uniq, inv = np.unique(np.concatenate(lists), return_inverse=True)
        twod = decode_records(proj.rec[torch.from_numpy(uniq.astype(np.int64)).cuda()].cpu().numpy())
        twod = (twod[0], twod[1], twod[2], twod[3], twod[4])
        rg_sub = np.zeros_like(rg, dtype=np.uint32)
        off = 0
        for t, l in zip(ts, lists):
            rg_sub[toff[v] + t] = (off, off + len(l))
            off += len(l)
        mask = np.zeros(cam.n_tiles, np.uint8)
        mask[ts] = 1
        ref = oracle.render_view(cam, oracle_opt(opts), int(toff[v]), twod, inv.astype(np.uint32), rg_sub,
                                 tile_mask=mask, guard_eps=oracle.STAGE_GUARD)
        where = np.zeros((cam.height, cam.width), bool)
        for t in ts:
            where[(t // cam.tiles_x) * 16:(t // cam.tiles_x + 1) * 16, (t % cam.tiles_x) * 16:(t % cam.tiles_x + 1) * 16] = True
        g = {k: imgs[k][v] for k in ("rgb", "depth", "alpha")}
        # the sampled tiles include each view's longest list, where decisions
        # near the skip / stop thresholds concentrate
        check_image(cam, oracle_opt(opts), int(toff[v]), twod, inv.astype(np.uint32), rg_sub, ref, g,
                    f"C5 view {v} sampled tiles", guard_eps=oracle.STAGE_GUARD, where=where, cap=1e-3)
