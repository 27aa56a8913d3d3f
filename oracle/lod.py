"""Level-of-detail selection for a served view, written from the paper.

TEST INFRASTRUCTURE ONLY (imported by ``tests/``).  Plain Python, double
precision, no shared code with the library.

Paper: §3.4.2 ("Detail Level Selection") chooses a level for every
render-time partition from the distance between the partition and the
camera, finer levels for closer partitions, and culls partitions the view
cannot see (Fig. 3b); the distance-threshold ablation (Tab. 13) gives each
level's threshold as the largest distance at which that level is used.

Readings where the paper is silent:
  * distance = from the camera centre to the nearest point of the
    partition's axis-aligned box (0 inside it);
  * visible = the box, grown by a margin on every side, is not entirely on
    the outer side of any one of the five frustum planes: z = near, and
    x = u z, y = v z at the image border widened by 15 % of the image size
    per side (the clamp of the projection's Jacobian);
  * budget (a choice of this library; the paper's budget caps training):
    while the total exceeds it, the farthest partition (ties: lower id) among
    those at the finest level still above 1 drops one level; when every kept
    partition is at level 1, the farthest is dropped; an error when even the
    last (nearest) partition does not fit.
"""
from __future__ import annotations

import math

import numpy as np


class BudgetError(ValueError):
    pass


def camera_centre(viewmat) -> np.ndarray:
    vm = np.asarray(viewmat, np.float64)
    return -vm[:3, :3].T @ vm[:3, 3]


def border_ratios(cam):
    """(u_lo, u_hi, v_lo, v_hi): image border widened by 15 % per side, as x/z and y/z."""
    W, H = float(cam.width), float(cam.height)
    return (-(cam.cx + 0.15 * W) / cam.fx, (W - cam.cx + 0.15 * W) / cam.fx,
            -(cam.cy + 0.15 * H) / cam.fy, (H - cam.cy + 0.15 * H) / cam.fy)


def in_view(cam, lo, hi, margin: float) -> bool:
    vm = np.asarray(cam.viewmat, np.float64)
    lo = np.asarray(lo, np.float64) - margin
    hi = np.asarray(hi, np.float64) + margin
    ulo, uhi, vlo, vhi = border_ratios(cam)
    near = float(getattr(cam, "near", 0.01))
    outside = [True] * 5
    for i in range(8):
        x = np.array([hi[0] if i & 1 else lo[0], hi[1] if i & 2 else lo[1], hi[2] if i & 4 else lo[2]])
        p = vm[:3, :3] @ x + vm[:3, 3]
        g = (p[2] - near, p[0] - ulo * p[2], uhi * p[2] - p[0], p[1] - vlo * p[2], vhi * p[2] - p[1])
        outside = [o and v < 0.0 for o, v in zip(outside, g)]
    return not any(outside)


def box_distance(c, lo, hi) -> float:
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    e = np.maximum(np.maximum(lo - c, 0.0), c - hi)
    return float(math.sqrt(float((e * e).sum())))


def level_for_distance(d: float, thresholds) -> int:
    """Finest level L for d <= thresholds[0], L - 1 for d <= thresholds[1], ..., 1 beyond."""
    n_levels = len(thresholds)
    for k, t in enumerate(thresholds):
        if d <= t:
            return n_levels - k
    return 1


def select(part_min, part_max, counts, thresholds, margin, cam, budget):
    """-> (levels [P] int, total).  counts [L][P]; level 0 = not drawn."""
    counts = np.asarray(counts, np.int64)
    n_parts = counts.shape[1]
    c = camera_centre(cam.viewmat)
    level = [0] * n_parts
    dist = [0.0] * n_parts
    for p in range(n_parts):
        if in_view(cam, part_min[p], part_max[p], margin):
            dist[p] = box_distance(c, part_min[p], part_max[p])
            level[p] = level_for_distance(dist[p], thresholds)
    visible = any(l > 0 for l in level)

    def total():
        return int(sum(counts[l - 1, p] for p, l in enumerate(level) if l > 0))

    def farthest(cands):
        return max(cands, key=lambda p: (dist[p], -p))

    while total() > budget:
        above = [p for p in range(n_parts) if level[p] > 1]
        if above:
            top = max(level[p] for p in above)
            p = farthest([q for q in above if level[q] == top])
            level[p] -= 1
        else:
            kept = [p for p in range(n_parts) if level[p] == 1]
            if not kept:
                break
            level[farthest(kept)] = 0
    if visible and not any(l > 0 for l in level):
        raise BudgetError("the budget cannot hold the nearest visible partition")
    return np.array(level, np.int32), total()
