"""All-pixels x all-Gaussians FP64 brute force, written independently of
``oracle.c`` in vectorised NumPy.  TEST INFRASTRUCTURE ONLY.

It follows the same readings of the paper (§3.1, Eq. 1 and Eq. 2) but is
organised the other way round: every Gaussian is projected at once, and
every pixel tests every Gaussian's tile rectangle instead of walking a
sorted per-tile list.  Meant for images up to 64x64 and a few hundred
Gaussians.
"""
from __future__ import annotations

import math

import numpy as np

TILE = 16


def _real_sh(d: np.ndarray, degree: int) -> np.ndarray:
    """Real SH basis from the spherical coordinates of unit directions,
    via associated Legendre functions computed by recurrence (the
    Condon-Shortley phase included), m = -l..l per band."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    theta = np.arccos(np.clip(z, -1.0, 1.0))
    phi = np.arctan2(y, x)
    ct = np.cos(theta)
    st = np.sin(theta)
    out = np.zeros((d.shape[0], 16))
    # P[l][m] for m >= 0 with the Condon-Shortley phase
    P = {}
    P[(0, 0)] = np.ones_like(ct)
    for m in range(1, 4):
        P[(m, m)] = -(2 * m - 1) * st * P[(m - 1, m - 1)]
    for m in range(0, 4):
        if m + 1 <= 3:
            P[(m + 1, m)] = (2 * m + 1) * ct * P[(m, m)]
        for l in range(m + 2, 4):
            P[(l, m)] = ((2 * l - 1) * ct * P[(l - 1, m)] - (l + m - 1) * P[(l - 2, m)]) / (l - m)
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            if m == 0:
                val = norm * P[(l, 0)]
            elif m > 0:
                val = math.sqrt(2.0) * norm * P[(l, am)] * np.cos(am * phi)
            else:
                val = math.sqrt(2.0) * norm * P[(l, am)] * np.sin(am * phi)
            out[:, l * l + l + m] = val
    return out


def _quat_rot(q: np.ndarray) -> np.ndarray:
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0] = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1)
    R[:, 1] = np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1)
    R[:, 2] = np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1)
    return R


def render(scene, cam, sh_degree=3, dilation=0.3, aa=False, bg=(0.0, 0.0, 0.0)) -> dict:
    mu = scene.means.T.astype(np.float64)
    s = scene.scales.T.astype(np.float64)
    q = scene.quats.T.astype(np.float64)
    o = scene.opacities.astype(np.float64)
    sh = scene.sh.astype(np.float64)                     # (16, 3, N)
    vm = np.asarray(cam.viewmat, np.float32).astype(np.float64)
    Rw, tw = vm[:3, :3], vm[:3, 3]
    fx, fy = float(np.float32(cam.fx)), float(np.float32(cam.fy))
    cx, cy = float(np.float32(cam.cx)), float(np.float32(cam.cy))
    W, H = cam.width, cam.height
    dil = float(np.float32(dilation))
    near, far = float(np.float32(cam.near)), float(np.float32(cam.far))

    t = mu @ Rw.T + tw
    tz = t[:, 2]
    ok = (tz >= near) & (tz <= far)
    tzs = np.where(ok, tz, 1.0)
    Rq = _quat_rot(q)
    Sig = Rq @ (s[:, :, None] ** 2 * np.transpose(Rq, (0, 2, 1)))
    u, v = t[:, 0] / tzs, t[:, 1] / tzs
    uc = np.clip(u, -(cx + 0.15 * W) / fx, (W - cx + 0.15 * W) / fx)
    vc = np.clip(v, -(cy + 0.15 * H) / fy, (H - cy + 0.15 * H) / fy)
    J = np.zeros((len(o), 2, 3))
    J[:, 0, 0] = fx / tzs
    J[:, 0, 2] = -fx * uc / tzs
    J[:, 1, 1] = fy / tzs
    J[:, 1, 2] = -fy * vc / tzs
    Tm = J @ Rw
    S2 = Tm @ Sig @ np.transpose(Tm, (0, 2, 1))
    a, b, c = S2[:, 0, 0], 0.5 * (S2[:, 0, 1] + S2[:, 1, 0]), S2[:, 1, 1]
    ad, cd = a + dil, c + dil
    detd = ad * cd - b * b
    det2 = a * c - b * b
    ok &= detd > 0
    rho = np.sqrt(np.clip(det2 / np.where(detd > 0, detd, 1.0), 0.0, None)) if aa else np.ones_like(o)
    A, B, Cc = cd / np.where(ok, detd, 1.0), -b / np.where(ok, detd, 1.0), ad / np.where(ok, detd, 1.0)
    mx, my = fx * u + cx, fy * v + cy
    lmax = 0.5 * (ad + cd) + np.sqrt(0.25 * (ad - cd) ** 2 + b * b)
    r = np.ceil(3.0 * np.sqrt(np.where(ok, lmax, 0.0)))
    TW, TH = (W + TILE - 1) // TILE, (H + TILE - 1) // TILE
    tx0 = np.maximum(0, np.floor((np.floor(mx) - r) / TILE))
    tx1 = np.minimum(TW - 1, np.floor((np.floor(mx) + r) / TILE))
    ty0 = np.maximum(0, np.floor((np.floor(my) - r) / TILE))
    ty1 = np.minimum(TH - 1, np.floor((np.floor(my) + r) / TILE))
    ok &= (tx0 <= tx1) & (ty0 <= ty1)

    campos = -Rw.T @ tw
    d = mu - campos
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = _real_sh(d, sh_degree)
    nb = (sh_degree + 1) ** 2
    raw = np.einsum("nk,kcn->nc", Y[:, :nb], sh[:nb]) + 0.5
    col = np.maximum(raw, 0.0)
    op = o * rho
    key = tz.astype(np.float32).view(np.uint32)

    idx = np.nonzero(ok)[0]
    order = idx[np.lexsort((idx, key[idx]))]             # depth key, then index
    rgb = np.zeros((H, W, 3))
    dep = np.zeros((H, W))
    T = np.ones((H, W))
    last = np.zeros((H, W), np.int32)
    for py in range(H):
        for px in range(W):
            ptx, pty = px // TILE, py // TILE
            cover = order[(tx0[order] <= ptx) & (ptx <= tx1[order]) & (ty0[order] <= pty) & (pty <= ty1[order])]
            Tp, C3, D, lst = 1.0, np.zeros(3), 0.0, 0
            for pos, g in enumerate(cover):
                dx, dy = px + 0.5 - mx[g], py + 0.5 - my[g]
                power = -0.5 * (A[g] * dx * dx + Cc[g] * dy * dy) - B[g] * dx * dy
                if power > 0:
                    continue
                al = min(0.99, op[g] * math.exp(power))
                if al < 1.0 / 255.0:
                    continue
                Tn = Tp * (1.0 - al)
                if Tn < 1e-4:
                    break
                C3 += col[g] * al * Tp
                D += tz[g] * al * Tp
                Tp = Tn
                lst = pos + 1
            rgb[py, px] = C3 + Tp * np.asarray(bg, np.float64)
            dep[py, px] = D
            T[py, px] = Tp
            last[py, px] = lst
    return {"rgb": rgb, "depth": dep, "alpha": 1.0 - T, "T": T, "last": last}
