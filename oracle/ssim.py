"""D-SSIM term of the training loss, written from the paper.

TEST INFRASTRUCTURE ONLY (imported by ``tests/``).  Double precision NumPy,
no shared code with the library.

Paper: Eq. 3 combines the L1 term with a D-SSIM term weighted by lambda =
0.2, taken from 3DGS.  Readings: SSIM of Wang et al. per pixel and channel
over an 11x11 Gaussian window (sigma 1.5, weights normalised to 1), values
outside the image taken as 0, C1 = 0.01^2 and C2 = 0.03^2 (unit dynamic
range); D-SSIM = 1 - the mean of the SSIM map over pixels and channels.
The gradient is the chain rule through the window means (the window is
symmetric, so its adjoint is the same zero-padded blur).
"""
from __future__ import annotations

import numpy as np

C1, C2 = 0.01 ** 2, 0.03 ** 2
RADIUS = 5


def window() -> np.ndarray:
    d = np.arange(-RADIUS, RADIUS + 1, dtype=np.float64)
    w = np.exp(-d * d / (2.0 * 1.5 * 1.5))
    return w / w.sum()


def blur(img: np.ndarray) -> np.ndarray:
    """Separable correlation of each channel of [H, W, C] with the window,
    zero outside the image."""
    w = window()
    H, W = img.shape[:2]
    p = np.pad(img, ((RADIUS, RADIUS), (RADIUS, RADIUS), (0, 0)))
    rows = sum(w[k] * p[:, k:k + W] for k in range(2 * RADIUS + 1))
    return sum(w[k] * rows[k:k + H] for k in range(2 * RADIUS + 1))


def ssim_map(x: np.ndarray, y: np.ndarray):
    mx, my = blur(x), blur(y)
    bx2, by2, bxy = blur(x * x), blur(y * y), blur(x * y)
    vx, vy, cxy = bx2 - mx * mx, by2 - my * my, bxy - mx * my
    A1, A2 = 2 * mx * my + C1, 2 * cxy + C2
    B1, B2 = mx * mx + my * my + C1, vx + vy + C2
    return A1 * A2 / (B1 * B2), (mx, my, A1, A2, B1, B2)


def dssim(rgb, target, weight=0.2):
    """-> (weight * (1 - mean SSIM), gradient w.r.t. rgb), float64; images [H, W, 3]."""
    x = np.asarray(rgb, np.float64)
    y = np.asarray(target, np.float64)
    s, (mx, my, A1, A2, B1, B2) = ssim_map(x, y)
    n = s.size
    loss = weight * (1.0 - s.mean())
    den = B1 * B2
    # partial derivatives of s w.r.t. a = G*x, b = G*(x^2), c = G*(xy)
    pa = (2 * my * (A2 - A1) - s * 2 * mx * (B2 - B1)) / den
    pb = -s / B2
    pc = 2 * A1 / den
    grad = -(weight / n) * (blur(pa) + 2 * x * blur(pb) + y * blur(pc))
    return float(loss), grad
