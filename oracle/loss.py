"""Training loss of the rasterizer path, written from the paper.

TEST INFRASTRUCTURE ONLY (imported by ``tests/``).  Double precision NumPy,
no shared code with the library.

Paper: the L1 term of Eq. 3 between the rendered and the captured image, and
the depth regulariser of §3.5.3 (weight lambda_d, initial value 0.5 in §3.6)
as an L1 distance on the expected depth.  Reading: expected depth = rendered
depth D / alpha with alpha clamped below at 1e-10; |x| is differentiated as
sign(x) (0 at 0); the clamp passes no gradient below 1e-10.  The D-SSIM term
of Eq. 3 is not part of this loss.
"""
from __future__ import annotations

import numpy as np


def l1_depth(rgb, depth, alpha, target_rgb, target_depth=None, lambda_depth=0.5):
    """-> (loss, d_rgb, d_depth, d_alpha), all float64; rgb [P, 3], the rest [P]."""
    rgb = np.asarray(rgb, np.float64)
    t_rgb = np.asarray(target_rgb, np.float64)
    n = rgb.shape[0]
    e = rgb - t_rgb
    loss = np.abs(e).sum() / (3.0 * n)
    d_rgb = np.sign(e) / (3.0 * n)
    d_depth = np.zeros(n)
    d_alpha = np.zeros(n)
    if target_depth is not None:
        D = np.asarray(depth, np.float64)
        a = np.asarray(alpha, np.float64)
        clamped = ~(a >= 1e-10)
        am = np.where(clamped, 1e-10, a)
        ed = D / am - np.asarray(target_depth, np.float64)
        loss += lambda_depth * np.abs(ed).sum() / n
        s = lambda_depth * np.sign(ed) / n
        d_depth = s / am
        d_alpha = np.where(clamped, 0.0, -s * D / (am * am))
    return float(loss), d_rgb, d_depth, d_alpha
