"""MI355X (gfx950) differentiable 3D-Gaussian tile rasterizer.

The hot path -- projection, SH colour, tile binning and sort, compositing of
colour and depth, and the backward -- runs in the HIP kernels of libgs.so
behind the C ABI of include/gs.h, as do the level-of-detail selection and
the batching server for rendering requests, the appearance transform MLP
whose offsets the rasterizer applies, and the densification bookkeeping and
3D smoothing filter that consume the backward's statistics.  This package only marshals torch tensors
(device memory, streams) into that ABI; it has no CPU fallback.
"""
from ._lib import GsError, load, LIB_PATH
from .rasterizer import (RenderOptions, RenderStats, Projected, Workspace, GsRasterize, rasterize, project,
                         bin_sort, render_fwd, render_bwd, seg_workspace, split_views, views_extent, grad2d_view, check_params, set_stage_hook, render_count,
                         kernel_timing, kernel_timing_read, L1DepthLoss, l1_depth_loss, DSSIMLoss, dssim_loss)
from .serving import LodTable, lod_select, ServeConfig, Server
from . import densify
from .appearance import AppearanceParams, AppearanceOffsets, appearance_offsets, mlp_fwd as appearance_mlp_fwd, mlp_bwd as appearance_mlp_bwd


def build(verbose: bool = False) -> str:
    from .build import build as _build
    return _build(verbose)


__all__ = ["GsError", "load", "LIB_PATH", "RenderOptions", "RenderStats", "Projected", "Workspace", "GsRasterize",
           "rasterize", "project", "bin_sort", "render_fwd", "render_bwd", "seg_workspace", "split_views", "views_extent",
           "grad2d_view", "check_params", "set_stage_hook", "render_count", "kernel_timing", "kernel_timing_read", "build", "L1DepthLoss", "l1_depth_loss", "DSSIMLoss", "dssim_loss", "LodTable", "lod_select",
           "ServeConfig", "Server", "AppearanceParams", "AppearanceOffsets", "appearance_offsets",
           "appearance_mlp_fwd", "appearance_mlp_bwd", "densify"]
