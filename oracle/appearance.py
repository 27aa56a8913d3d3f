"""FP64 oracle of the appearance transform module (§3.5.1, Fig. "appearance
transform"; sizes from the implementation details of the appendix).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, never by the GPU library.

Per Gaussian i, the module maps its own embedding (16 values) and the
image's embedding (32 values) through one hidden layer of 32 ReLU units and
a sigmoid output layer of 4 units to colour and opacity offsets
(dc_r, dc_g, dc_b, do).  Readings where the text is silent:

* "normalized embeddings are used" (the similarity regulariser's premise):
  both embeddings enter the MLP divided by max(|l|, 1e-12);
* input order: the Gaussian embedding first, then the image embedding;
  W1 is [32][48], W2 is [4][32];
* the sigmoid outputs are offsets around the identity: colour
  c' = max(0, SH(d) + dc) = max(0, c + dc - 1/2) (dc = 1/2 leaves it
  unchanged) and opacity o' = o (1 - do) (do = 0 leaves it unchanged, which
  is what the opacity-offset regulariser's minimisation of mean do drives
  towards);
* the opacity-offset regulariser is L = lambda * mean_i do_i.

Gradients are written out by the chain rule (no automatic differentiation)
so that a finite-difference test pins them independently.
"""
from __future__ import annotations

import numpy as np

GAUSS_DIM, IMAGE_DIM, HIDDEN, OUT = 16, 32, 32, 4
EPS = 1e-12


def _normalise(v):
    nrm = np.sqrt((v * v).sum(-1, keepdims=True))
    den = np.maximum(nrm, EPS)
    return v / den, den, nrm > EPS


def _normalise_bwd(vhat, den, above, dvhat):
    """Gradient through v / max(|v|, eps): (dv_hat - v_hat (v_hat . dv_hat)) / |v|
    above the floor, dv_hat / eps at it."""
    dot = (vhat * dvhat).sum(-1, keepdims=True)
    proj = np.where(above, dvhat - vhat * dot, dvhat)
    return proj / den


def mlp_forward(gemb, iemb, w1, b1, w2, b2) -> dict:
    """gemb [n][16], iemb [32], w1 [32][48], b1 [32], w2 [4][32], b2 [4] ->
    dict with y [n][4] (the offsets) and the intermediates."""
    g = np.asarray(gemb, np.float64).reshape(-1, GAUSS_DIM)
    e = np.asarray(iemb, np.float64).reshape(IMAGE_DIM)
    w1 = np.asarray(w1, np.float64).reshape(HIDDEN, GAUSS_DIM + IMAGE_DIM)
    b1 = np.asarray(b1, np.float64).reshape(HIDDEN)
    w2 = np.asarray(w2, np.float64).reshape(OUT, HIDDEN)
    b2 = np.asarray(b2, np.float64).reshape(OUT)
    ghat, gden, gabove = _normalise(g)
    ehat, eden, eabove = _normalise(e[None, :])
    x = np.concatenate([ghat, np.broadcast_to(ehat, (g.shape[0], IMAGE_DIM))], 1)
    a = x @ w1.T + b1
    h = np.maximum(a, 0.0)
    z = h @ w2.T + b2
    y = 1.0 / (1.0 + np.exp(-z))
    return {"y": y, "x": x, "a": a, "h": h, "z": z, "ghat": ghat, "gden": gden, "gabove": gabove,
            "ehat": ehat[0], "eden": eden[0], "eabove": eabove[0], "w1": w1, "w2": w2}


def mlp_backward(fwd: dict, dy, reg_weight: float = 0.0) -> dict:
    """Gradients of sum(dy * y) + reg_weight * mean(y[:, 3]) with respect to
    every input of mlp_forward."""
    y, x, a, h = fwd["y"], fwd["x"], fwd["a"], fwd["h"]
    w1, w2 = fwd["w1"], fwd["w2"]
    n = y.shape[0]
    dy = np.array(dy, np.float64).reshape(n, OUT)
    if n:
        dy[:, 3] += reg_weight / n
    dz = dy * y * (1.0 - y)
    d_w2 = dz.T @ h
    d_b2 = dz.sum(0)
    dh = dz @ w2
    da = dh * (a > 0.0)
    d_w1 = da.T @ x
    d_b1 = da.sum(0)
    dx = da @ w1
    d_gemb = _normalise_bwd(fwd["ghat"], fwd["gden"], fwd["gabove"], dx[:, :GAUSS_DIM])
    de_hat = dx[:, GAUSS_DIM:].sum(0)
    d_iemb = _normalise_bwd(fwd["ehat"][None, :], fwd["eden"][None, :], fwd["eabove"][None, :],
                            de_hat[None, :])[0]
    return {"gemb": d_gemb, "iemb": d_iemb, "w1": d_w1, "b1": d_b1, "w2": d_w2, "b2": d_b2}


def opacity_reg(y, reg_weight: float) -> float:
    """lambda * mean of the opacity offsets (0 for no Gaussians)."""
    y = np.asarray(y, np.float64).reshape(-1, OUT)
    return float(reg_weight * y[:, 3].mean()) if y.shape[0] else 0.0


def apply_offsets(opacities, y):
    """Opacity and colour base seen by the rasterizer under offsets y:
    o' = o (1 - do); the colour base replaces the SH +1/2 by dc."""
    y = np.asarray(y, np.float64).reshape(-1, OUT)
    return np.asarray(opacities, np.float64) * (1.0 - y[:, 3]), np.ascontiguousarray(y[:, :3])


def apply_offsets_bwd(opacities, y, d_opac_eff, d_colour_base):
    """Chains the rasterizer's gradients with respect to o' and the colour
    base to (d opacities, d y)."""
    y = np.asarray(y, np.float64).reshape(-1, OUT)
    o = np.asarray(opacities, np.float64)
    d_o = d_opac_eff * (1.0 - y[:, 3])
    dy = np.zeros_like(y)
    dy[:, :3] = d_colour_base
    dy[:, 3] = -d_opac_eff * o
    return d_o, dy
