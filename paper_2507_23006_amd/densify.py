"""Densification bookkeeping and the 3D smoothing filter (include/gs.h,
gs_densify_* and gs_filter3d_*): marshalling of torch tensors into the
library's kernels.

  accumulate(stats, tiles, ...)   running statistic of the backward's
                                  per-view |dL/d mean2d| (or AbsGS sums)
  select(stats, params, ...)      per-Gaussian action under Eq. 4's
                                  in-partition thresholds and a budget
  filter3d_rate / filter3d        Mip-Splatting 3D smoothing filter
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L
from .rasterizer import Workspace, _check_param, _default_ws, _ptr, _stream

KEEP, CLONE, SPLIT, PRUNE = 0, 1, 2, 3


class DensifyStats:
    """Running sum and view count per Gaussian (float32 / int32, on the GPU)."""

    def __init__(self, n: int, device):
        self.accum = torch.zeros(n, dtype=torch.float32, device=device)
        self.count = torch.zeros(n, dtype=torch.int32, device=device)

    def reset(self) -> None:
        self.accum.zero_()
        self.count.zero_()


def accumulate(st: DensifyStats, tiles, grad_norm=None, absgrad=None, view_scale=None) -> None:
    """Adds one step: tiles [V*n] or [V, n] (int32 tile counts of the
    projection), grad_norm [V, n] or absgrad [V, n, 2]; view_scale: V floats."""
    lib = L.load()
    n = st.accum.shape[0]
    V = tiles.numel() // n
    if tiles.numel() != V * n or (grad_norm is None) == (absgrad is None):
        raise ValueError("tiles must hold V * n counts and exactly one of grad_norm / absgrad is given")
    tiles = tiles.contiguous()
    g = grad_norm.contiguous() if grad_norm is not None else None
    a = absgrad.contiguous() if absgrad is not None else None
    if g is not None:
        _check_param(g, "grad_norm", (V, n))
    if a is not None:
        _check_param(a, "absgrad", (V, n, 2))
    sc = None
    if view_scale is not None:
        sc = (C.c_float * V)(*[float(x) for x in view_scale])
    L.check(lib.gs_densify_accumulate(_ptr(tiles), _ptr(g), _ptr(a), V, n, sc, _ptr(st.accum), _ptr(st.count),
                                      _stream()))


@dataclass
class DensifyParams:
    box_min: tuple
    box_max: tuple
    tau_min: float = 2e-4
    eta: float = 4.0
    d_max: float = 100.0
    prune_opacity: float = 0.005
    split_scale: float = 0.1
    budget: int = 0

    def c(self) -> L.GsDensifyParams:
        p = L.GsDensifyParams()
        for k in range(3):
            p.box_min[k], p.box_max[k] = float(self.box_min[k]), float(self.box_max[k])
        p.tau_min, p.eta, p.d_max = float(self.tau_min), float(self.eta), float(self.d_max)
        p.prune_opacity, p.split_scale, p.budget = float(self.prune_opacity), float(self.split_scale), int(self.budget)
        return p


def select(st: DensifyStats, means, scales, opacities, params: DensifyParams):
    """-> (action uint8 [n] (KEEP/CLONE/SPLIT/PRUNE), counts dict)."""
    lib = L.load()
    n = st.accum.shape[0]
    _check_param(means, "means", (3, n))
    _check_param(scales, "scales", (3, n))
    _check_param(opacities, "opacities", (n,))
    action = torch.empty(n, dtype=torch.uint8, device=means.device)
    counts = (C.c_int64 * 4)()
    wsz = lib.gs_densify_workspace_size(n)
    ws = _default_ws.get("densify", wsz + 256, means.device)
    pc = params.c()
    L.check(lib.gs_densify_select(_ptr(st.accum), _ptr(st.count), _ptr(means), _ptr(scales), _ptr(opacities), n,
                                  C.byref(pc), _ptr(action), counts, C.c_void_p(Workspace.aligned(ws)), wsz,
                                  _stream()))
    return action, {"candidates": counts[0], "pruned": counts[1], "grown": counts[2], "room": counts[3]}


def filter3d_rate(means, cams) -> torch.Tensor:
    """Sampling rate [n] of every mean over the cameras (0 where none sees it)."""
    lib = L.load()
    n = means.shape[-1]
    _check_param(means, "means", (3, n))
    rate = torch.empty(n, dtype=torch.float32, device=means.device)
    cams = list(cams)
    L.check(lib.gs_filter3d_rate(_ptr(means), n, L.make_cameras(cams), len(cams), _ptr(rate), _stream()))
    return rate


class Filter3D(torch.autograd.Function):
    """(scales [3, n], opacities [n]) -> 3D-filtered (scales', opacities')
    for fixed rates [n] and filter size s_f."""

    @staticmethod
    def forward(ctx, scales, opacities, rate, s_f: float):
        lib = L.load()
        n = opacities.shape[0]
        scales, opacities, rate = scales.detach().contiguous(), opacities.detach().contiguous(), rate.detach().contiguous()
        _check_param(scales, "scales", (3, n))
        _check_param(rate, "rate", (n,))
        s2, o2 = torch.empty_like(scales), torch.empty_like(opacities)
        L.check(lib.gs_filter3d_fwd(_ptr(scales), _ptr(opacities), _ptr(rate), n, float(s_f), _ptr(s2), _ptr(o2),
                                    _stream()))
        ctx.save_for_backward(scales, opacities, rate)
        ctx.s_f = float(s_f)
        return s2, o2

    @staticmethod
    def backward(ctx, d_s2, d_o2):
        lib = L.load()
        scales, opacities, rate = ctx.saved_tensors
        n = opacities.shape[0]
        d_s2 = torch.zeros_like(scales) if d_s2 is None else d_s2.contiguous()
        d_o2 = torch.zeros_like(opacities) if d_o2 is None else d_o2.contiguous()
        ds, do = torch.empty_like(scales), torch.empty_like(opacities)
        L.check(lib.gs_filter3d_bwd(_ptr(scales), _ptr(opacities), _ptr(rate), n, ctx.s_f, _ptr(d_s2), _ptr(d_o2),
                                    _ptr(ds), _ptr(do), _stream()))
        return ds, do, None, None


def filter3d(scales, opacities, rate, s_f: float):
    return Filter3D.apply(scales, opacities, rate, s_f)
