"""FP64 oracle of the densification bookkeeping that consumes the
rasterizer's backward statistics.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, never by the GPU library.

Paper passages: the mean image-space gradient that 3DGS densification
thresholds (§3.1, after Eq. 2); the absolute-gradient variant (AbsGS,
§3.5.4); the in-partition threshold of Eq. 4 (§3.3) with eta = 4 and d_max =
the partition size (appendix); the Gaussian budget B of the steerable
densification each detail level is trained under (§3.4.1); the 3D smoothing
filter of the Mip-Splatting anti-aliasing (§3.5.4).

Readings where the text is silent (the same in the kernels):
* statistic per view where the Gaussian was rasterized (tiles > 0):
  |dL/d mean2d| times a per-view scale (pixel -> NDC units, or 1), or, in the
  AbsGS mode, |(sum_p |dL_p/dx|, sum_p |dL_p/dy|)| times that scale; summed
  over views and iterations with a count of views; mean = sum / count in
  double precision (the plain quotient; a compared float32 implementation
  differs from it only by rounding, which a test absorbs by setting aside
  decisions within that rounding of their boundary);
* d_i = Euclidean distance from the mean to the partition's axis-aligned box
  (0 inside); tau_i = tau_min (min(d_i, d_max) / d_max (eta - 1) + 1) (Eq. 4);
  a Gaussian is a candidate when its mean exceeds tau_i;
* pruning (opacity below a floor) is decided first and excludes densifying;
* budget cap: at most K = max(0, B - (n - n_pruned)) candidates are kept,
  those with the largest mean / tau_i (ties: lower index);
* a kept candidate is split when its largest scale exceeds a threshold, else
  cloned (the 3DGS rule);
* 3D filter: the sampling rate of Gaussian i is nu_i = max over cameras whose
  view holds its mean (depth in [near, far], projection within the image
  extent widened by 15 % per side) of f_x / depth; the filter adds
  sigma^2 = (s_f / nu_i)^2 to every axis of Sigma (no filter when no camera
  sees it).  Because sigma^2 I commutes with the rotation, scales become
  sqrt(s^2 + sigma^2) and the opacity is compensated by
  sqrt(det Sigma / det Sigma') = prod_k s_k / s'_k.
"""
from __future__ import annotations

import numpy as np

KEEP, CLONE, SPLIT, PRUNE = 0, 1, 2, 3


def accumulate(tiles, grad_norm=None, absgrad=None, view_scale=None, accum=None, count=None):
    """tiles [V][n]; grad_norm [V][n] or absgrad [V][n][2] -> (accum, count)
    after adding this step's views (new arrays when none are given)."""
    tiles = np.asarray(tiles)
    V, n = tiles.shape
    acc = np.zeros(n) if accum is None else np.array(accum, np.float64)
    cnt = np.zeros(n, np.int64) if count is None else np.array(count, np.int64)
    sc = np.ones(V) if view_scale is None else np.asarray(view_scale, np.float64)
    for v in range(V):
        if absgrad is not None:
            a = np.asarray(absgrad, np.float64)[v]
            val = np.sqrt(a[:, 0] ** 2 + a[:, 1] ** 2)
        else:
            val = np.asarray(grad_norm, np.float64)[v]
        seen = tiles[v] > 0
        acc[seen] += val[seen] * sc[v]
        cnt[seen] += 1
    return acc, cnt


def box_distance(means, box_min, box_max):
    """Distance of each mean [3][n] to the axis-aligned box (0 inside)."""
    m = np.asarray(means, np.float64)
    lo = np.asarray(box_min, np.float64)[:, None]
    hi = np.asarray(box_max, np.float64)[:, None]
    d = np.maximum(np.maximum(lo - m, m - hi), 0.0)
    return np.sqrt((d * d).sum(0))


def thresholds(means, box_min, box_max, tau_min, eta, d_max):
    """tau_i of Eq. 4 and d_i."""
    d = box_distance(means, box_min, box_max)
    return tau_min * (np.minimum(d, d_max) / d_max * (eta - 1.0) + 1.0), d


def select(accum, count, means, scales, opacities, box_min, box_max, tau_min, eta, d_max, prune_opacity,
           split_scale, budget):
    """Actions [n] (KEEP/CLONE/SPLIT/PRUNE) and the intermediate values."""
    acc = np.asarray(accum, np.float64)
    cnt = np.asarray(count, np.int64)
    n = acc.shape[0]
    mean = np.where(cnt > 0, acc / np.maximum(cnt, 1), 0.0)
    tau, d = thresholds(means, box_min, box_max, tau_min, eta, d_max)
    prune = np.asarray(opacities, np.float64) < prune_opacity
    cand = (mean > tau) & ~prune
    score = np.where(cand, mean / tau, 0.0)
    k = max(0, int(budget) - (n - int(prune.sum())))
    idx = np.nonzero(cand)[0]
    order = sorted(idx.tolist(), key=lambda i: (-score[i], i))
    kept = np.array(order[:k], np.int64)
    act = np.zeros(n, np.uint8)
    act[prune] = PRUNE
    big = np.asarray(scales, np.float64).max(0) > split_scale
    act[kept] = np.where(big[kept], SPLIT, CLONE)
    return {"action": act, "mean": mean, "tau": tau, "d": d, "score": score, "k": k, "candidates": idx,
            "kept": kept}


def filter_rate(means, cams):
    """nu_i = max over cameras that see the mean of f_x / depth (0 if none)."""
    m = np.asarray(means, np.float64)
    rate = np.zeros(m.shape[1])
    for c in cams:
        vm = np.asarray(c.viewmat, np.float32).astype(np.float64)
        t = vm[:3, :3] @ m + vm[:3, 3:4]
        z = t[2]
        fx, fy = float(np.float32(c.fx)), float(np.float32(c.fy))
        cx, cy = float(np.float32(c.cx)), float(np.float32(c.cy))
        W, H = c.width, c.height
        with np.errstate(divide="ignore", invalid="ignore"):
            # the mean is in front and its image-plane ratios x / z, y / z lie
            # within the image extent widened by 15 % of the size per side
            u, v = t[0] / z, t[1] / z
            ok = (z >= float(np.float32(c.near))) & (z <= float(np.float32(c.far)))
            ok &= (u >= -(cx + 0.15 * W) / fx) & (u <= (W - cx + 0.15 * W) / fx)
            ok &= (v >= -(cy + 0.15 * H) / fy) & (v <= (H - cy + 0.15 * H) / fy)
            r = np.where(ok, fx / z, 0.0)
        rate = np.maximum(rate, r)
    return rate


def filter_rate_margin(means, cams):
    """Per Gaussian, the smallest relative distance of a camera's view test
    (depth against near / far, x / z and y / z against the widened image
    bounds) from its boundary: decisions this close to their boundary can go
    either way under rounding and are set aside by comparisons."""
    m = np.asarray(means, np.float64)
    out = np.full(m.shape[1], np.inf)
    for c in cams:
        vm = np.asarray(c.viewmat, np.float32).astype(np.float64)
        t = vm[:3, :3] @ m + vm[:3, 3:4]
        z = t[2]
        fx, fy = float(np.float32(c.fx)), float(np.float32(c.fy))
        cx, cy = float(np.float32(c.cx)), float(np.float32(c.cy))
        W, H = c.width, c.height
        near, far = float(np.float32(c.near)), float(np.float32(c.far))
        with np.errstate(divide="ignore", invalid="ignore"):
            u, v = t[0] / z, t[1] / z
            for val, b in ((z, near), (z, far), (u, -(cx + 0.15 * W) / fx), (u, (W - cx + 0.15 * W) / fx),
                           (v, -(cy + 0.15 * H) / fy), (v, (H - cy + 0.15 * H) / fy)):
                d = np.abs(val - b) / max(1.0, abs(b))
                out = np.minimum(out, np.where(np.isfinite(d), d, np.inf))
    return out


def filter_apply(scales, opacities, rate, s_f):
    """(scales' [3][n], opacities' [n]) of the 3D-filtered Gaussians."""
    s = np.asarray(scales, np.float64)
    o = np.asarray(opacities, np.float64)
    r = np.asarray(rate, np.float64)
    var = np.where(r > 0, (s_f / np.where(r > 0, r, 1.0)) ** 2, 0.0)
    s2 = np.sqrt(s * s + var)
    return s2, o * np.prod(s / s2, axis=0)


def filter_bwd(scales, opacities, rate, s_f, d_scales_out, d_opac_out):
    """Chain rule of filter_apply: (d scales [3][n], d opacities [n])."""
    s = np.asarray(scales, np.float64)
    o = np.asarray(opacities, np.float64)
    r = np.asarray(rate, np.float64)
    var = np.where(r > 0, (s_f / np.where(r > 0, r, 1.0)) ** 2, 0.0)
    s2 = np.sqrt(s * s + var)
    comp = np.prod(s / s2, axis=0)
    o2 = o * comp
    ds = np.asarray(d_scales_out, np.float64) * s / s2            # through s' = sqrt(s^2 + var)
    ds += np.asarray(d_opac_out, np.float64) * o2 * var / (s * s2 * s2)   # d log(s/s')/ds = var / (s s'^2)
    return ds, np.asarray(d_opac_out, np.float64) * comp
