"""Synthetic scenes and cameras with the shapes of the paper's urban workloads.

The paper measures on aerial and street-level captures of city blocks
(millions of Gaussians, images up to 1600 px on the long edge, §4.1 and
Supp. A).  Those captures and the trained scenes are not available, so
every workload here is drawn from fixed distributions with a fixed seed.

Conventions (shared by every consumer of these arrays):

* World is z-up.  Cameras use OpenCV axes: x right, y down, z forward.
* ``viewmat`` is the 4x4 world-to-camera matrix [R | t; 0 0 0 1].
* Gaussian parameters are structure-of-arrays, float32:
  ``means[3][N]``, ``scales[3][N]`` (already exponentiated, > 0),
  ``quats[4][N]`` as (w, x, y, z), ``opacities[N]`` (already passed
  through a sigmoid), ``sh[16][3][N]`` (coefficient, channel, Gaussian).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SH_COEFFS = 16


@dataclass
class Camera:
    fx: float
    fy: float
    cx: float
    cy: float
    viewmat: np.ndarray          # (4, 4) float32, world -> camera
    width: int
    height: int
    near: float = 0.01
    far: float = 1e10

    @property
    def tiles_x(self) -> int:
        return (self.width + 15) // 16

    @property
    def tiles_y(self) -> int:
        return (self.height + 15) // 16

    @property
    def n_tiles(self) -> int:
        return self.tiles_x * self.tiles_y

    @property
    def n_pixels(self) -> int:
        return self.width * self.height


@dataclass
class Scene:
    means: np.ndarray        # (3, N)
    scales: np.ndarray       # (3, N)
    quats: np.ndarray        # (4, N)
    opacities: np.ndarray    # (N,)
    sh: np.ndarray           # (16, 3, N)

    @property
    def n(self) -> int:
        return int(self.opacities.shape[0])

    def param_arrays(self) -> list:
        """The five parameter arrays as contiguous float32 in the layout the
        rasterizer library takes: the colour coefficients as one row per
        Gaussian, (N, 16, 3); the others as stored."""
        return [np.ascontiguousarray(a, dtype=np.float32)
                for a in (self.means, self.scales, self.quats, self.opacities, self.sh.transpose(2, 0, 1))]

    def subset(self, idx: np.ndarray) -> "Scene":
        return Scene(np.ascontiguousarray(self.means[:, idx]),
                     np.ascontiguousarray(self.scales[:, idx]),
                     np.ascontiguousarray(self.quats[:, idx]),
                     np.ascontiguousarray(self.opacities[idx]),
                     np.ascontiguousarray(self.sh[:, :, idx]))


@dataclass
class LodScene:
    """Levels 1 (coarsest) .. L (finest) of one scene, each stored
    partition-major so that every (level, partition) is one contiguous
    range, plus the render-time partition table."""
    levels: list                       # list[Scene], coarsest first
    part_min: np.ndarray               # (P, 3) float32 AABB min
    part_max: np.ndarray               # (P, 3) float32 AABB max
    offsets: np.ndarray                # (L, P) int64 start within level
    counts: np.ndarray                 # (L, P) int64
    thresholds: tuple = (30.0, 60.0, math.inf)   # finest level used up to d0, ...
    extra: dict = field(default_factory=dict)

    def combined(self):
        """All levels in one parameter set (coarsest first) and the start of
        every (level, partition) range in it: (Scene, offsets (L, P) int64)."""
        base = np.concatenate([[0], np.cumsum([lv.n for lv in self.levels])[:-1]]).astype(np.int64)
        cat = lambda name, axis: np.ascontiguousarray(
            np.concatenate([getattr(lv, name) for lv in self.levels], axis=axis))
        sc = Scene(cat("means", 1), cat("scales", 1), cat("quats", 1), cat("opacities", 0), cat("sh", 2))
        return sc, self.offsets + base[:, None]


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------

def look_at(eye, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """World-to-camera matrix for an OpenCV camera at ``eye`` looking at
    ``target`` with world ``up`` (default z-up)."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    rot = np.stack([r, d, f], 0)
    m = np.eye(4)
    m[:3, :3] = rot
    m[:3, 3] = -rot @ eye
    return m.astype(np.float32)


def pose_camera(eye, yaw, pitch, width, height, hfov_deg=70.0) -> Camera:
    fwd = np.array([math.cos(pitch) * math.cos(yaw),
                    math.cos(pitch) * math.sin(yaw),
                    math.sin(pitch)])
    vm = look_at(eye, np.asarray(eye) + fwd)
    f = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    return Camera(float(np.float32(f)), float(np.float32(f)), width / 2.0, height / 2.0,
                  vm, width, height)


def camera_c1() -> Camera:
    """160x120 pinhole, fx=fy=150, camera centre at z=-4 looking along +z."""
    vm = np.eye(4, dtype=np.float32)
    vm[2, 3] = 4.0
    return Camera(150.0, 150.0, 80.0, 60.0, vm, 160, 120)


def camera_c2() -> Camera:
    """1600x1066 camera 30 m above the block, looking 60 deg down at the origin."""
    w, h = 1600, 1066
    f = float(np.float32((w / 2.0) / math.tan(math.radians(35.0))))
    vm = look_at((0.0, -17.32, 30.0), (0.0, 0.0, 0.0))
    return Camera(f, f, w / 2.0, h / 2.0, vm, w, h)


def camera_c3(seed: int = 2) -> Camera:
    """1920x1080 street-level camera at 1.7 m, heading +x, pitched 5 deg down,
    with a small seeded jitter so that no axis is exactly aligned."""
    rng = np.random.default_rng(seed)
    eye = np.array([0.0, 0.0, 1.7]) + rng.normal(0.0, 0.02, 3)
    yaw = math.radians(rng.normal(0.0, 0.2))
    pitch = math.radians(-5.0 + rng.normal(0.0, 0.2))
    return pose_camera(eye, yaw, pitch, 1920, 1080)


def cameras_c5() -> list:
    """Eight views on the street path, alternating heading, mixed resolutions:
    two 3840x2160, three 1920x1080, three 1280x720."""
    res = [(3840, 2160)] * 2 + [(1920, 1080)] * 3 + [(1280, 720)] * 3
    cams = []
    for k in range(8):
        x = -87.5 + 25.0 * k
        yaw = 0.0 if k % 2 == 0 else math.pi
        cams.append(pose_camera((x, 0.0, 1.7), yaw, math.radians(-5.0), *res[k]))
    return cams


# --------------------------------------------------------------------------
# scenes
# --------------------------------------------------------------------------

def _attributes(rng, n, log_scale_mu, log_scale_sigma):
    scales = np.exp(rng.normal(log_scale_mu, log_scale_sigma, (3, n))).astype(np.float32)
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    quats = q.astype(np.float32)
    opac = (1.0 / (1.0 + np.exp(-rng.standard_normal(n)))).astype(np.float32)
    sh = rng.standard_normal((SH_COEFFS, 3, n), dtype=np.float32)
    sh[0] *= np.float32(0.5)
    sh[1:] *= np.float32(0.05)
    return scales, quats, opac, sh


def random_scene(n: int, seed: int, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0),
                 log_scale_mu=-3.0, log_scale_sigma=0.5) -> Scene:
    """Means uniform in a box; log-scales normal; random unit quaternions;
    sigmoid(N(0,1)) opacities; SH DC ~ N(0, 0.5), higher bands ~ N(0, 0.05)."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, np.float64)[:, None]
    hi = np.asarray(hi, np.float64)[:, None]
    means = (lo + (hi - lo) * rng.random((3, n))).astype(np.float32)
    scales, quats, opac, sh = _attributes(rng, n, log_scale_mu, log_scale_sigma)
    return Scene(means, scales, quats, opac, sh)


def scene_c1(seed: int = 0) -> Scene:
    return random_scene(4096, seed)


def scene_c2(seed: int = 0) -> Scene:
    return random_scene(1_000_000, seed, lo=(-20.0, -20.0, 0.0), hi=(20.0, 20.0, 10.0))


def scene_urban(n: int, n_boxes: int, seed: int = 0, extent: float = 150.0) -> Scene:
    """Urban block: 70% of the Gaussians on a noisy ground plane over
    [-extent, extent]^2, 30% on the vertical faces of axis-aligned boxes
    (buildings) that leave a street corridor |y| <= 12 m free."""
    rng = np.random.default_rng(seed)
    n_ground = int(round(0.7 * n))
    n_facade = n - n_ground
    means = np.empty((3, n), np.float64)
    means[0, :n_ground] = rng.uniform(-extent, extent, n_ground)
    means[1, :n_ground] = rng.uniform(-extent, extent, n_ground)
    means[2, :n_ground] = rng.normal(0.0, 0.1, n_ground)

    # building boxes: centre (x, y) with |y| > 12, half widths, heights
    cx = rng.uniform(-extent + 10.0, extent - 10.0, n_boxes)
    cy = np.empty(n_boxes)
    filled = 0
    while filled < n_boxes:
        cand = rng.uniform(-extent + 10.0, extent - 10.0, 2 * n_boxes)
        cand = cand[np.abs(cand) > 12.0]
        take = min(len(cand), n_boxes - filled)
        cy[filled:filled + take] = cand[:take]
        filled += take
    hx = rng.uniform(3.0, 10.0, n_boxes)
    hy = rng.uniform(3.0, 10.0, n_boxes)
    hz = rng.uniform(6.0, 40.0, n_boxes)
    # faces: 0 (+x), 1 (-x) of area 2*hy*h; 2 (+y), 3 (-y) of area 2*hx*h
    face_area = np.stack([2 * hy * hz, 2 * hy * hz, 2 * hx * hz, 2 * hx * hz], 1)
    p_face = (face_area / face_area.sum()).ravel()
    pick = rng.choice(4 * n_boxes, size=n_facade, p=p_face)
    b, f = pick // 4, pick % 4
    s = rng.uniform(-1.0, 1.0, n_facade)           # position along the face
    hgt = rng.uniform(0.0, 1.0, n_facade) * hz[b]  # height on the face
    jit = rng.normal(0.0, 0.05, n_facade)          # jitter along the face normal
    x = np.where(f == 0, cx[b] + hx[b] + jit,
        np.where(f == 1, cx[b] - hx[b] - jit, cx[b] + s * hx[b]))
    y = np.where(f == 2, cy[b] + hy[b] + jit,
        np.where(f == 3, cy[b] - hy[b] - jit, cy[b] + s * hy[b]))
    means[0, n_ground:] = x
    means[1, n_ground:] = y
    means[2, n_ground:] = hgt
    scales, quats, opac, sh = _attributes(rng, n, -2.5, 0.7)
    return Scene(means.astype(np.float32), scales, quats, opac, sh)


def scene_c3(seed: int = 0) -> Scene:
    return scene_urban(6_000_000, 200, seed)


# --------------------------------------------------------------------------
# LOD stand-in and the serving trace
# --------------------------------------------------------------------------

def _hash_u64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (a public integer hash) used only to rank
    Gaussians inside a partition for the synthetic coarser levels."""
    z = x.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def lod_scene_c4(fine: Scene, part_size: float = 30.0, extent: float = 150.0,
                 fractions=(1.0 / 6.0, 0.5, 1.0)) -> LodScene:
    """Coarser levels as hash-ranked subsets of the finest level inside each
    render-time partition, with scales grown by sqrt(1/fraction) so that the
    surface stays covered.  A stand-in for trained LOD levels."""
    n_side = int(round(2 * extent / part_size))
    n_parts = n_side * n_side
    ix = np.clip(((fine.means[0].astype(np.float64) + extent) // part_size).astype(np.int64), 0, n_side - 1)
    iy = np.clip(((fine.means[1].astype(np.float64) + extent) // part_size).astype(np.int64), 0, n_side - 1)
    pid = iy * n_side + ix
    h = _hash_u64(np.arange(fine.n, dtype=np.uint64))
    order = np.lexsort((h, pid))             # partition-major, hash-ranked inside
    pid_sorted = pid[order]
    counts_fine = np.bincount(pid_sorted, minlength=n_parts)
    starts_fine = np.concatenate([[0], np.cumsum(counts_fine)[:-1]])
    rank = np.arange(fine.n) - starts_fine[pid_sorted]
    levels, offsets, counts = [], [], []
    for frac in fractions:
        keep_n = np.ceil(counts_fine * frac).astype(np.int64)
        keep = rank < keep_n[pid_sorted]
        idx = order[keep]
        lvl = fine.subset(idx)
        if frac < 1.0:
            lvl.scales *= np.float32(math.sqrt(1.0 / frac))
        levels.append(lvl)
        counts.append(keep_n)
        offsets.append(np.concatenate([[0], np.cumsum(keep_n)[:-1]]))
    gx = np.arange(n_side) * part_size - extent
    pmin = np.zeros((n_parts, 3), np.float32)
    pmax = np.zeros((n_parts, 3), np.float32)
    zs_min = np.full(n_parts, np.inf)
    zs_max = np.full(n_parts, -np.inf)
    np.minimum.at(zs_min, pid, fine.means[2])
    np.maximum.at(zs_max, pid, fine.means[2])
    zs_min[~np.isfinite(zs_min)] = 0.0
    zs_max[~np.isfinite(zs_max)] = 0.0
    for p in range(n_parts):
        px, py = p % n_side, p // n_side
        pmin[p] = (gx[px], gx[py], zs_min[p])
        pmax[p] = (gx[px] + part_size, gx[py] + part_size, zs_max[p])
    return LodScene(levels, pmin, pmax, np.stack(offsets), np.stack(counts))


def serve_trace_c4(n_requests: int = 2000, rate: float = 150.0, seed: int = 3):
    """Open-loop request trace: Poisson arrivals, random street poses on the
    200 m path, resolution and Gaussian budget drawn uniformly."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    res_choices = [(640, 360), (1280, 720), (1920, 1080)]
    budgets = [1_000_000, 3_000_000, 6_000_000]
    reqs = []
    for i in range(n_requests):
        s = rng.uniform(0.0, 1.0)
        eye = (-100.0 + 200.0 * s, 0.0, 1.7)
        yaw = rng.uniform(0.0, 2 * math.pi)
        pitch = math.radians(rng.uniform(-10.0, 5.0))
        w, h = res_choices[rng.integers(0, 3)]
        budget = budgets[rng.integers(0, 3)]
        reqs.append({"t": float(arrivals[i]), "camera": pose_camera(eye, yaw, pitch, w, h),
                     "budget": int(budget)})
    return reqs


# --------------------------------------------------------------------------
# targets and loss weights
# --------------------------------------------------------------------------

def target_rgb(height: int, width: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).random((height, width, 3), dtype=np.float32)


def target_depth(height: int, width: int, seed: int, lo=20.0, hi=45.0) -> np.ndarray:
    rng = np.random.default_rng(seed + 1000)
    return (lo + (hi - lo) * rng.random((height, width))).astype(np.float32)


def linear_loss_weights(height: int, width: int, seed: int = 7):
    """Weights of the linear test functional sum(w_rgb*rgb) + sum(w_d*depth)
    + sum(w_a*alpha); its upstream gradients are exactly the weights."""
    rng = np.random.default_rng(seed)
    w_rgb = rng.standard_normal((height, width, 3)).astype(np.float32)
    w_d = rng.standard_normal((height, width)).astype(np.float32)
    w_a = rng.standard_normal((height, width)).astype(np.float32)
    return w_rgb, w_d, w_a
