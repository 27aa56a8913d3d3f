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
