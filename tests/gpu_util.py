"""Helpers shared by the GPU tests: move seeded scenes to the device, run the
GPU path through the C ABI binding, and convert its records for the oracle.
Test infrastructure only."""
import math

import numpy as np
import torch

import oracle

LOG2E = 1.0 / math.log(2.0)


def to_dev(scene, device="cuda:0", requires_grad=False):
    ts = [torch.from_numpy(a).to(device) for a in scene.param_arrays()]
    if requires_grad:
        for t in ts:
            t.requires_grad_(True)
    return ts


def grads_oracle_layout(params):
    """Parameter gradients of GPU tensors as float64 arrays in the oracle's
    layouts (the colour coefficients back to (16, 3, N))."""
    g = {k: p.grad.cpu().numpy().astype(np.float64) for k, p in
         zip(("means", "scales", "quats", "opacities", "sh"), params)}
    g["sh"] = np.ascontiguousarray(g["sh"].transpose(1, 2, 0))
    return g


def decode_records(rec: np.ndarray):
    """GPU records [S, 16] -> oracle 2D quantities (float64, exact widening):
    mean2d (integer part + fraction), conic (A, B, C) undoing the -log2(e) (1/2, 1, 1/2) scaling,
    opacity', rgb, depth."""
    rec = rec.astype(np.float64)
    mean2d = np.stack([rec[:, 0] + rec[:, 7], rec[:, 1] + rec[:, 11]], 1)
    conic = np.stack([-2.0 * rec[:, 2] / LOG2E, -rec[:, 3] / LOG2E, -2.0 * rec[:, 4] / LOG2E], 1)
    return mean2d, conic, rec[:, 5].copy(), rec[:, 8:11].copy(), rec[:, 6].copy()


def mask_rows(mask: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Rows of a rectangle of width w spanned by the covered-tile bits of
    mask (0 where mask is 0)."""
    mask = np.asarray(mask).view(np.uint64)
    hi, lo = (mask >> np.uint64(32)).astype(np.float64), (mask & np.uint64(0xFFFFFFFF)).astype(np.float64)
    # highest set bit: frexp's exponent is exact for integers below 2^53
    top = np.where(hi > 0, 31 + np.frexp(hi)[1], np.frexp(lo)[1] - 1).astype(np.int64)
    return np.where(mask != 0, top // np.maximum(w, 1) + 1, 0)


def mask_covers(mask, w, x0, y0, tx, ty) -> np.ndarray:
    """For slots with a covered-tile mask (0 = every tile of the rectangle):
    whether tile (tx, ty) is covered, given it lies in the rectangle."""
    mask = np.asarray(mask).view(np.uint64)
    bit = np.clip((ty - y0) * w + (tx - x0), 0, 63).astype(np.uint64)
    return (mask == 0) | (((mask >> bit) & np.uint64(1)) == 1)


def decode_rect(rect: np.ndarray, tiles: np.ndarray, cams, n, mask=None):
    """GPU rect words -> (tile x0, y0, x1, y1) per slot, view-local.  With
    exact tile culling (mask != 0) the height is the last row holding a
    covered tile (rows below hold none)."""
    rect = rect.view(np.uint32).astype(np.int64)
    tiles = tiles.astype(np.int64)
    out = np.zeros((len(tiles), 4), np.int64)
    toff = np.cumsum([0] + [c.n_tiles for c in cams])[:-1]
    for v, c in enumerate(cams):
        sl = slice(v * n, (v + 1) * n)
        base = rect[sl, 0] - toff[v]
        w = rect[sl, 1] & 0xFFFF
        tw = rect[sl, 1] >> 16
        vis = tiles[sl] > 0
        x0 = np.where(vis, base % c.tiles_x, 0)
        y0 = np.where(vis, base // c.tiles_x, 0)
        h = np.where(vis, tiles[sl] // np.maximum(w, 1), 0)
        if mask is not None:
            mv = np.asarray(mask).view(np.uint64)[sl]
            h = np.where(vis & (mv != 0), mask_rows(mv, w), h)
        out[sl] = np.stack([x0, y0, x0 + w - 1, y0 + h - 1], 1) * vis[:, None]
        assert np.all(tw[vis] == c.tiles_x)
    return out


def gpu_forward(gs, scene, cams, opts):
    params = to_dev(scene)
    n = scene.n
    proj = gs.project(*params, cams, opts)
    pairs, ranges, P = gs.bin_sort(proj, cams, n)
    out = gs.render_fwd(proj, pairs, ranges, cams, opts)
    torch.cuda.synchronize()
    return params, proj, pairs, ranges, P, out


def oracle_opt(opts):
    return dict(sh_degree=opts.sh_degree, dilation=opts.dilation, aa=opts.aa, bg=opts.bg)


def view_images(flat, cams):
    out, off = [], 0
    for c in cams:
        k = c.width * c.height
        out.append(flat[off:off + k].reshape(c.height, c.width, *flat.shape[1:]))
        off += k
    return out


def border_slots(projs):
    """Slots whose 3-sigma rectangle rests on a value within rounding of an
    integer (the extent 3 sqrt(lambda_max), or the mean's pixel index): a
    float32 and an FP64 rectangle may differ by one there."""
    out = []
    for p in projs:
        out.append((p["tiles"] > 0) & ((np.abs(p["extent"] - np.round(p["extent"])) < 1e-9) |
                                       np.any(np.abs(p["mean2d"] - np.round(p["mean2d"])) < 1e-9, axis=1)))
    return np.concatenate(out)


def gpu_pair_ids(pairs, ranges, P, n_slots):
    """(global tile) * n_slots + slot of every GPU pair, in list order."""
    rg = ranges.cpu().numpy().view(np.uint32).astype(np.int64)
    pv = pairs.cpu().numpy().view(np.uint32)[:P].astype(np.int64)
    tile = np.repeat(np.arange(len(rg)), rg[:, 1] - rg[:, 0])
    assert len(tile) == P
    return tile * n_slots + pv


def check_tile_culling(f, pairs, ranges, P):
    """Tile culling of the GPU path against the oracle's definition of it
    (oracle.bin_pairs with ``reach``: a tile is needed where the FP64 record
    passes the skip rule at some pixel centre).  ``f`` is an unculled
    oracle.forward of the same scene and cameras.  Every needed (tile, slot)
    pair must be among the GPU's pairs and every GPU pair must lie in the
    oracle's 3-sigma rectangle, slots on a rounding border aside.  Returns
    (needed, gpu, extra): the GPU pairs beyond the needed ones are the price
    of its conservative per-tile test."""
    cams = f["cams"]
    n_slots = len(f["bins"]["tiles"])
    rect = np.concatenate([p["rect"] for p in f["proj"]])
    tiles = np.concatenate([p["tiles"] for p in f["proj"]])
    keys = oracle.depth_key(np.concatenate([p["depth"] for p in f["proj"]]))
    n = len(f["proj"][0]["tiles"])
    sv = np.repeat(np.arange(len(cams), dtype=np.int32), n)
    need = oracle.bin_pairs(rect, tiles, keys, sv, cams, reach=f["twod"][:3])
    full = f["bins"]
    assert full["n_pairs"] == int(tiles.astype(np.int64).sum()), "f must be an unculled forward"
    ids_need = need["pair_tile"].astype(np.int64) * n_slots + need["pair_slot"]
    ids_full = full["pair_tile"].astype(np.int64) * n_slots + full["pair_slot"]
    ids_gpu = gpu_pair_ids(pairs, ranges, P, n_slots)
    border = border_slots(f["proj"])
    sl_need = need["pair_slot"].astype(np.int64)
    missing = ~np.isin(ids_need, ids_gpu) & ~border[sl_need]
    assert not missing.any(), f"{int(missing.sum())} needed pairs missing, e.g. slot {sl_need[missing][:5]}"
    outside = ~np.isin(ids_gpu, ids_full) & ~border[ids_gpu % n_slots]
    assert not outside.any(), f"{int(outside.sum())} GPU pairs outside the 3-sigma rectangles"
    extra = int((~np.isin(ids_gpu, ids_need)).sum())
    return need["n_pairs"], P, extra


# Pixels with more flagged decisions than compare_image enumerates (2^4
# alternatives) stay unchecked; their share of an image is capped here.
UNRESOLVED_CAP = 1e-4


def check_image(cam, opt: dict, tile_off: int, twod, pair_slot, ranges, ref: dict, got: dict, label: str = "",
                guard_eps=oracle.DEFAULT_GUARD, cap: float = UNRESOLVED_CAP, where=None) -> dict:
    """One view of a GPU image against the oracle's render over the same
    lists: max |d| <= 1e-4 on rgb and alpha and <= 1e-4 max(1, depth) on the
    accumulated depth outside the guard band; inside it, a match with one of
    the results the pixel's flagged decisions allow (oracle.compare_image).
    Prints the counts; asserts no mismatch and at most ``cap`` of the
    pixels unresolved.  ``where`` (bool [H][W]) limits it to some pixels."""
    r = oracle.compare_image(cam, opt, tile_off, twod, pair_slot, ranges, ref, got, guard_eps=guard_eps, where=where)
    n_px = cam.n_pixels if where is None else int(np.count_nonzero(where))
    print(f"{label}: worst {r['worst']:.2e} outside the guard band; {r['flagged']} of {n_px} pixels flagged "
          f"({r['flagged'] / n_px:.1e}), {r['resolved']} matched an alternative, {r['unresolved']} unresolved, "
          f"{r['mismatch']} mismatched", flush=True)
    assert r["worst"] <= 1e-4, (label, r)
    assert r["mismatch"] == 0, (label, r)
    assert r["unresolved"] <= cap * n_px, (label, r)
    return r


def compare_grad(got, ref, name, rel_tol=1e-3):
    """Gradient parity of one group: ||g - g_ref|| / ||g_ref|| <= rel_tol, and
    |g - g_ref| <= 1e-3 |g_ref| + 1e-3 rms(g_ref) for >= 99.9 % of entries.
    Returns the relative error."""
    a, b = np.asarray(got, np.float64).ravel(), np.asarray(ref, np.float64).ravel()
    nb = np.linalg.norm(b)
    assert nb > 0, name
    rel = np.linalg.norm(a - b) / nb
    assert rel <= rel_tol, (name, rel)
    rms = np.sqrt(np.mean(b * b))
    good = np.abs(a - b) <= 1e-3 * np.abs(b) + 1e-3 * rms
    assert good.mean() >= 0.999, (name, good.mean())
    return rel


def linear_loss(ws, rgb, depth, alpha):
    """sum of w_rgb rgb + w_d depth + w_a alpha over the views' pixels (the
    views' weight arrays concatenated in view order)."""
    w_rgb = torch.from_numpy(np.concatenate([w[0].reshape(-1, 3) for w in ws])).cuda()
    w_d = torch.from_numpy(np.concatenate([w[1].reshape(-1) for w in ws])).cuda()
    w_a = torch.from_numpy(np.concatenate([w[2].reshape(-1) for w in ws])).cuda()
    return (w_rgb * rgb).sum() + (w_d * depth).sum() + (w_a * alpha).sum()
