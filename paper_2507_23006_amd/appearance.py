"""Appearance transform module (§3.5.1): per-Gaussian colour and opacity
offsets from a Gaussian embedding [N, 16] and an image embedding [32]
through a small MLP (48 -> 32 ReLU -> 4 sigmoid), as an autograd Function
over the library's matrix-core kernels (include/gs.h, gs_appearance_*).

The offsets feed ``rasterize(..., app=offsets)``.  They depend only on the
embeddings and the MLP, so a renderer computes them once per image
embedding and reuses them for every frame."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L
from .rasterizer import Workspace, _check_param, _default_ws, _ptr, _stream

GAUSS_DIM, IMAGE_DIM, HIDDEN, OUT = 16, 32, 32, 4


@dataclass
class AppearanceParams:
    """MLP weights: w1 [32, 48] (Gaussian-embedding columns first), b1 [32],
    w2 [4, 32], b2 [4]."""
    w1: torch.Tensor
    b1: torch.Tensor
    w2: torch.Tensor
    b2: torch.Tensor

    @staticmethod
    def init(device, seed: int = 0, scale: float = 0.3) -> "AppearanceParams":
        g = torch.Generator(device="cpu").manual_seed(seed)
        mk = lambda *s: (torch.randn(*s, generator=g) * scale).to(device)
        return AppearanceParams(mk(HIDDEN, GAUSS_DIM + IMAGE_DIM), mk(HIDDEN), mk(OUT, HIDDEN), mk(OUT))


def _mlp_struct(w1, b1, w2, b2) -> L.GsAppearanceMlp:
    m = L.GsAppearanceMlp()
    m.w1, m.b1, m.w2, m.b2 = w1.data_ptr(), b1.data_ptr(), w2.data_ptr(), b2.data_ptr()
    return m


def _check_mlp(image_emb, w1, b1, w2, b2):
    ins = [t.detach().contiguous() for t in (image_emb, w1, b1, w2, b2)]
    for t, name, shape in zip(ins, ("image_emb", "w1", "b1", "w2", "b2"),
                              ((IMAGE_DIM,), (HIDDEN, GAUSS_DIM + IMAGE_DIM), (HIDDEN,), (OUT, HIDDEN), (OUT,))):
        _check_param(t, name, shape)
    return ins


def mlp_fwd(gauss_emb, image_emb, w1, b1, w2, b2, reg_weight: float = 0.0):
    """gs_appearance_fwd: (offsets [N, 4], reg [1] = reg_weight * mean do)."""
    lib = L.load()
    gemb = gauss_emb.detach().contiguous()
    n = gemb.shape[0]
    _check_param(gemb, "gauss_emb", (n, GAUSS_DIM))
    iemb, w1, b1, w2, b2 = _check_mlp(image_emb, w1, b1, w2, b2)
    dev = gemb.device
    offsets = torch.empty((n, OUT), dtype=torch.float32, device=dev)
    reg = torch.empty((1,), dtype=torch.float32, device=dev)
    wsz = lib.gs_appearance_workspace_size(n)
    ws = _default_ws.get("app", wsz + 256, dev)
    m = _mlp_struct(w1, b1, w2, b2)
    L.check(lib.gs_appearance_fwd(_ptr(gemb), n, _ptr(iemb), C.byref(m), float(reg_weight), _ptr(offsets),
                                  _ptr(reg), C.c_void_p(Workspace.aligned(ws)), wsz, _stream()))
    return offsets, reg


def mlp_bwd(gauss_emb, image_emb, w1, b1, w2, b2, offsets, d_offsets, d_reg=None, reg_weight: float = 0.0):
    """gs_appearance_bwd: (d_gauss_emb, d_image_emb, d_w1, d_b1, d_w2, d_b2)."""
    lib = L.load()
    gemb = gauss_emb.detach().contiguous()
    n = gemb.shape[0]
    _check_param(gemb, "gauss_emb", (n, GAUSS_DIM))
    iemb, w1, b1, w2, b2 = _check_mlp(image_emb, w1, b1, w2, b2)
    offsets, d_offsets = offsets.detach().contiguous(), d_offsets.detach().contiguous()
    _check_param(offsets, "offsets", (n, OUT))
    _check_param(d_offsets, "d_offsets", (n, OUT))
    if d_reg is not None:
        d_reg = d_reg.detach().reshape(1).contiguous()
        _check_param(d_reg, "d_reg", (1,))
    dev = gemb.device
    d_gemb = torch.empty_like(gemb)
    grads = [torch.empty_like(t) for t in (iemb, w1, b1, w2, b2)]
    go = L.GsAppearanceGrad()
    go.d_image_emb, go.d_w1, go.d_b1, go.d_w2, go.d_b2 = (t.data_ptr() for t in grads)
    wsz = lib.gs_appearance_workspace_size(n)
    ws = _default_ws.get("app", wsz + 256, dev)
    m = _mlp_struct(w1, b1, w2, b2)
    L.check(lib.gs_appearance_bwd(_ptr(gemb), n, _ptr(iemb), C.byref(m), _ptr(offsets), _ptr(d_offsets),
                                  _ptr(d_reg), float(reg_weight), _ptr(d_gemb), C.byref(go),
                                  C.c_void_p(Workspace.aligned(ws)), wsz, _stream()))
    return (d_gemb, *grads)


class AppearanceOffsets(torch.autograd.Function):
    """(gauss_emb, image_emb, w1, b1, w2, b2) -> (offsets [N, 4],
    reg_weight * mean of the opacity offsets)."""

    @staticmethod
    def forward(ctx, gauss_emb, image_emb, w1, b1, w2, b2, reg_weight: float):
        offsets, reg = mlp_fwd(gauss_emb, image_emb, w1, b1, w2, b2, reg_weight)
        ctx.save_for_backward(gauss_emb.detach(), image_emb.detach(), w1.detach(), b1.detach(), w2.detach(),
                              b2.detach(), offsets)
        ctx.reg_weight = float(reg_weight)
        return offsets, reg[0]

    @staticmethod
    def backward(ctx, d_offsets, d_reg):
        gemb, iemb, w1, b1, w2, b2, offsets = ctx.saved_tensors
        if d_offsets is None:
            d_offsets = torch.zeros_like(offsets)
        return (*mlp_bwd(gemb, iemb, w1, b1, w2, b2, offsets, d_offsets, d_reg, ctx.reg_weight), None)


def appearance_offsets(gauss_emb, image_emb, p: AppearanceParams, reg_weight: float = 0.0):
    """Returns (offsets [N, 4] = (dc_r, dc_g, dc_b, do), reg_weight * mean do)."""
    return AppearanceOffsets.apply(gauss_emb, image_emb, p.w1, p.b1, p.w2, p.b2, reg_weight)
