"""Torch-facing wrapper of libgs: device buffers and streams come from torch,
every computation runs in the library's gfx950 kernels.

Parameter layout (structure-of-arrays, float32, on the GPU):
  means [3, N], scales [3, N] (positive), quats [4, N] as (w, x, y, z),
  opacities [N] in (0, 1), sh [N, 16, 3]; optional appearance offsets
  app [N, 4] (see appearance.py).
Outputs of several views are concatenated per pixel (view-major, each view
row-major); ``split_views`` reshapes them into per-view images.
"""
from __future__ import annotations

import ctypes as C
import weakref
from dataclasses import dataclass

import torch

from . import _lib as L


@dataclass
class RenderOptions:
    sh_degree: int = 3
    dilation: float = 0.3
    aa: bool = False            # opacity compensation of the dilation (Mip-Splatting style 2D filter)
    bg: tuple = (0.0, 0.0, 0.0)
    absgrad: bool = False       # also accumulate |dL_p/d mean2d| per pixel (AbsGS)

    def c(self) -> L.GsOptions:
        return L.make_options(self.sh_degree, self.dilation, self.aa, self.bg)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_param(t: torch.Tensor, name: str, shape) -> None:
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def check_params(means, scales, quats, opacities, sh) -> int:
    n = means.shape[-1]
    _check_param(means, "means", (3, n))
    _check_param(scales, "scales", (3, n))
    _check_param(quats, "quats", (4, n))
    _check_param(opacities, "opacities", (n,))
    _check_param(sh, "sh", (n, 16, 3))
    return n


def check_app(app, n: int) -> None:
    if app is not None:
        _check_param(app, "app", (n, 4))


def gaussians_struct(means, scales, quats, opacities, sh, app=None) -> L.GsGaussians:
    g = L.GsGaussians()
    g.means, g.scales, g.quats = means.data_ptr(), scales.data_ptr(), quats.data_ptr()
    g.opacities, g.sh, g.n = opacities.data_ptr(), sh.data_ptr(), means.shape[-1]
    g.app = app.data_ptr() if app is not None else None
    return g


class Workspace:
    """Grow-only device scratch buffers, one per purpose (the library itself
    never allocates device memory)."""

    def __init__(self):
        self._bufs = {}
        self.pair_caps = {}      # (slots, tiles) -> pair capacity of gs_bin_sort

    def get(self, name: str, nbytes: int, device) -> torch.Tensor:
        b = self._bufs.get(name)
        if b is None or b.numel() < nbytes or b.device != device:
            b = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)
            self._bufs[name] = b
        return b

    @staticmethod
    def aligned(buf: torch.Tensor) -> int:
        p = buf.data_ptr()
        return (p + 255) & ~255


_default_ws = Workspace()


@dataclass
class Projected:
    rec: torch.Tensor        # [S, 16] float32
    rect: torch.Tensor       # [S, 2] int32 (bit patterns of uint32)
    tiles: torch.Tensor      # [S] int32
    depth_key: torch.Tensor  # [S] int32 (bit patterns of uint32)
    tile_order: torch.Tensor | None = None   # [T] int32, written by bin_sort
    tile_mask: torch.Tensor | None = None    # [S] int64 (bit patterns of uint64): exact tile culling

    def c(self) -> L.GsProjected:
        p = L.GsProjected()
        p.rec, p.rect = self.rec.data_ptr(), self.rect.data_ptr()
        p.tiles, p.depth_key = self.tiles.data_ptr(), self.depth_key.data_ptr()
        p.tile_order = self.tile_order.data_ptr() if self.tile_order is not None else None
        p.tile_mask = self.tile_mask.data_ptr() if self.tile_mask is not None else None
        return p


def views_extent(cams) -> tuple:
    lib = L.load()
    arr = L.make_cameras(cams)
    nt, npx = C.c_int64(), C.c_int64()
    L.check(lib.gs_views_extent(arr, len(cams), C.byref(nt), C.byref(npx)))
    return nt.value, npx.value


def project(means, scales, quats, opacities, sh, cams, opts: RenderOptions, app=None,
            exact_cull: bool = True) -> Projected:
    """exact_cull: per-tile ellipse culling (tile_mask); False keeps every
    tile of the alpha box's rectangle."""
    lib = L.load()
    n = check_params(means, scales, quats, opacities, sh)
    check_app(app, n)
    S = n * len(cams)
    dev = means.device
    n_tiles, _ = views_extent(cams)
    out = Projected(torch.empty((S, L.REC_FLOATS), dtype=torch.float32, device=dev),
                    torch.empty((S, 2), dtype=torch.int32, device=dev),
                    torch.empty((S,), dtype=torch.int32, device=dev),
                    torch.empty((S,), dtype=torch.int32, device=dev),
                    torch.empty((n_tiles,), dtype=torch.int32, device=dev),
                    torch.empty((S,), dtype=torch.int64, device=dev) if exact_cull else None)
    g = gaussians_struct(means, scales, quats, opacities, sh, app)
    L.check(lib.gs_project(C.byref(g), L.make_cameras(cams), len(cams), C.byref(opts.c()), C.byref(out.c()),
                           _stream()))
    return out


class _PinnedRing:
    """Pinned host slots for pair counts, taken round-robin, so that a loop
    that runs ahead of the device does not allocate pinned memory on every
    call.  A slot is reused only once the copy into it has completed; its
    previous count is then kept in its PairCount before the slot is
    overwritten (else a fresh pinned tensor is taken)."""

    SLOTS = 256

    def __init__(self):
        self.buf = torch.empty((self.SLOTS,), dtype=torch.int64, pin_memory=True)
        self.owners = [None] * self.SLOTS
        self.next = 0

    def take(self, pc: "PairCount"):
        i = self.next
        self.next = (i + 1) % self.SLOTS
        prev = self.owners[i]() if self.owners[i] is not None else None
        if prev is not None and prev._value is None:
            if not prev._event.query():
                return torch.empty((1,), dtype=torch.int64, pin_memory=True)
            prev._value = int(prev._host[0])
        self.owners[i] = weakref.ref(pc)
        return self.buf[i:i + 1]


_pinned_rings = {}


class PairCount:
    """The pair count of an asynchronous binning: the library writes it to
    device memory; int() waits for that write (a copy to pinned host memory
    queued behind the binning) and returns it.  A count above `capacity`
    means the binning produced empty tile lists and must be repeated with a
    larger pair buffer."""

    def __init__(self, dev_count: torch.Tensor, capacity: int):
        self.capacity = int(capacity)
        self._value = None
        key = dev_count.device.index or 0
        ring = _pinned_rings.get(key)
        if ring is None:
            ring = _pinned_rings[key] = _PinnedRing()
        self._event = torch.cuda.Event()
        self._host = ring.take(self)
        self._host.copy_(dev_count, non_blocking=True)
        self._event.record()

    def __int__(self) -> int:
        if self._value is None:
            self._event.synchronize()
            self._value = int(self._host[0])
        return self._value

    def overflowed(self) -> bool:
        return int(self) > self.capacity


def _pair_capacity(P: int) -> int:
    return int(P * 1.25) + 4096


def bin_sort(proj: Projected, cams, n: int, ws: Workspace | None = None, capacity_hint: int | None = None,
             sync: bool = True):
    """Returns (pair_vals, tile_ranges [T, 2] int32, P).  The library bins
    without any host read-back.  With sync (default) P is read here as an
    int -- the call is repeated with a larger pair buffer when P exceeded
    it -- and pair_vals is [P] (one unused element when P = 0).  With
    sync=False nothing waits: pair_vals is the whole capacity buffer and P a
    PairCount to check later.  pair_vals is a fresh tensor (torch's caching
    allocator), so results of several calls can be alive at once; the
    workspace remembers, per (slots, tiles), a capacity 25 % above the last
    count it read."""
    lib = L.load()
    ws = ws or _default_ws
    dev = proj.rec.device
    S = n * len(cams)
    n_tiles, _ = views_extent(cams)
    key = (S, n_tiles)
    cap = int(capacity_hint or ws.pair_caps.get(key, 0) or max(1 << 20, 4 * S))
    ranges = torch.empty((n_tiles, 2), dtype=torch.int32, device=dev)
    cams_c = L.make_cameras(cams)
    npairs = torch.empty((1,), dtype=torch.int64, device=dev)
    for _ in range(3):
        pairs = torch.empty((max(cap, 1),), dtype=torch.int32, device=dev)
        wsz = lib.gs_bin_workspace_size(S, cap)
        wbuf = ws.get("bin", wsz + 256, dev)
        L.check(lib.gs_bin_sort(C.byref(proj.c()), cams_c, len(cams), n, cap, _ptr(pairs), _ptr(ranges),
                                C.c_void_p(npairs.data_ptr()), C.c_void_p(Workspace.aligned(wbuf)), wsz, _stream()))
        if not sync:
            return pairs, ranges, PairCount(npairs, cap)
        P = int(npairs.item())
        if P > 0xFFFFFF00:
            raise L.GsError(L.GS_ERR_CAPACITY, f"{P} pairs exceed 32-bit indexing")
        ws.pair_caps[key] = _pair_capacity(P)
        if P > cap:
            cap = ws.pair_caps[key]
            continue
        # an empty view has a null data pointer in torch; with no pairs hand
        # back one (never read) element so the buffer pointer stays valid
        return (pairs[:P] if P > 0 else pairs[:1]), ranges, P
    raise L.GsError(L.GS_ERR_CAPACITY, "pair buffer could not be grown")


def seg_workspace(cams, pair_vals) -> torch.Tensor:
    """A device area for the segmented backward of these lists
    (gs_seg_workspace_size bytes, plus alignment slack)."""
    n_tiles, _ = views_extent(cams)
    ssz = L.load().gs_seg_workspace_size(n_tiles, int(pair_vals.numel()))
    return torch.empty(ssz + 256, dtype=torch.uint8, device=pair_vals.device)


def _seg_args(seg: torch.Tensor):
    base = Workspace.aligned(seg)
    return C.c_void_p(base), seg.numel() - (base - seg.data_ptr())


def render_fwd(proj: Projected, pair_vals, ranges, cams, opts: RenderOptions, seg=None, ws: Workspace | None = None) -> dict:
    """Compositing.  Lists longer than 512 positions are walked in segments
    by separate workgroups (gs_render_fwd_seg) in a workspace area; with
    `seg` (from seg_workspace) in that area, whose segment states the
    backward can then read (pass it to render_bwd).  seg=False: every list
    walked whole by one workgroup (gs_render_fwd)."""
    if seg is None:
        ws = ws or _default_ws
        n_tiles, _ = views_extent(cams)
        seg = ws.get("seg_fwd", L.load().gs_seg_workspace_size(n_tiles, int(pair_vals.numel())) + 256,
                     proj.rec.device)
    lib = L.load()
    dev = proj.rec.device
    _, npx = views_extent(cams)
    out = {"rgb": torch.empty((npx, 3), dtype=torch.float32, device=dev),
           "depth": torch.empty((npx,), dtype=torch.float32, device=dev),
           "alpha": torch.empty((npx,), dtype=torch.float32, device=dev),
           "T": torch.empty((npx,), dtype=torch.float32, device=dev),
           "last": torch.empty((npx,), dtype=torch.int32, device=dev)}
    args = (C.byref(proj.c()), _ptr(pair_vals), _ptr(ranges), L.make_cameras(cams), len(cams), C.byref(opts.c()),
            _ptr(out["rgb"]), _ptr(out["depth"]), _ptr(out["alpha"]), _ptr(out["T"]), _ptr(out["last"]))
    if seg is False:
        L.check(lib.gs_render_fwd(*args, _stream()))
    else:
        L.check(lib.gs_render_fwd_seg(*args, *_seg_args(seg), _stream()))
    return out


def render_count(proj: Projected, pair_vals, ranges, cams) -> torch.Tensor:
    """Per-pixel numbers of list entries the forward [:, 0] and the backward
    [:, 1] compositing evaluate (measurement)."""
    lib = L.load()
    _, npx = views_extent(cams)
    out = torch.empty((npx, 2), dtype=torch.int32, device=proj.rec.device)
    L.check(lib.gs_render_count(C.byref(proj.c()), _ptr(pair_vals), _ptr(ranges), L.make_cameras(cams), len(cams),
                                _ptr(out), _stream()))
    return out


KERNELS_TIMED = {"k_project_fwd": 0, "bin_sort": 1, "k_render_fwd": 2, "k_render_bwd": 3, "k_project_bwd": 4}


def kernel_timing(enable: bool) -> None:
    """Turns the library's per-launch event timing of the main kernels on or
    off (measurement); either way, pending measurements are dropped."""
    L.check(L.load().gs_kernel_timing(1 if enable else 0))


def kernel_timing_read(name: str):
    """(total ms, launches) of the timed launches of one kernel since the
    last read, measured with events on its own stream."""
    ms, k = C.c_double(), C.c_int64()
    L.check(L.load().gs_kernel_timing_read(KERNELS_TIMED[name], C.byref(ms), C.byref(k)))
    return ms.value, k.value


_stage_hook = None


def set_stage_hook(fn) -> None:
    """fn(name) is called on the host right after each stage is enqueued
    (project, bin_sort, render_fwd, composite_bwd, project_bwd); used by the
    benchmark to record stream events.  None disables it."""
    global _stage_hook
    _stage_hook = fn


def _mark(name: str) -> None:
    if _stage_hook is not None:
        _stage_hook(name)


_side_streams = {}


def _side_stream(dev) -> torch.cuda.Stream:
    """A second stream per device (default priority) for work that runs beside
    the main stream's."""
    key = torch.device(dev).index or 0
    if key not in _side_streams:
        _side_streams[key] = torch.cuda.Stream(device=dev)
    return _side_streams[key]


def _grad_struct(grads: dict) -> L.GsGaussiansGrad:
    go = L.GsGaussiansGrad()
    go.d_means, go.d_scales, go.d_quats = grads["means"].data_ptr(), grads["scales"].data_ptr(), grads["quats"].data_ptr()
    go.d_opacities, go.d_sh = grads["opacities"].data_ptr(), grads["sh"].data_ptr()
    if "app" in grads:
        go.d_app = grads["app"].data_ptr()
    return go


# Gaussian count from which the backward zeroes the gradient arrays on a
# second stream (below it the two cross-stream waits cost more than the
# fill saves)
FILL_BESIDE_MIN = 1 << 21


def _zeroed_grads(params, app, after: torch.cuda.Event, n: int):
    """Gradient arrays shaped like the parameters (and `app`), zeroed by
    gs_grads_zero on a second stream once the main stream has reached
    `after`, beside the main stream's next launches.  Returns (grads, event),
    the event recorded when they hold zeros."""
    lib = L.load()
    dev = params[0].device
    grads = {k: torch.empty_like(t) for k, t in zip(("means", "scales", "quats", "opacities", "sh"), params)}
    if app is not None:
        grads["app"] = torch.empty_like(app)
    side = _side_stream(dev)
    side.wait_event(after)
    # no record_stream: the caller's stream waits for `zeroed` before its
    # next launch, so the arrays (allocated on that stream, whose later
    # allocations alone can reuse their memory) are never reused under the
    # fill; recorded, their blocks would be held back from the allocator
    # until it saw the fill done, and a step allocating before that would
    # take fresh device memory
    L.check(lib.gs_grads_zero(C.byref(_grad_struct(grads)), n, C.c_void_p(side.cuda_stream)))
    zeroed = torch.cuda.Event()
    zeroed.record(side)
    return grads, zeroed


def render_bwd(params, cams, opts: RenderOptions, proj: Projected, pair_vals, ranges, T, last, d_rgb, d_depth,
               d_alpha, ws: Workspace | None = None, app=None, seg: torch.Tensor | None = None) -> dict:
    """Backward of compositing and projection; `seg`: the area the forward
    filled (render_fwd(..., seg=...)) for these lists, else the segment
    states are computed here."""
    lib = L.load()
    ws = ws or _default_ws
    means, scales, quats, opacities, sh = params
    n = check_params(means, scales, quats, opacities, sh)
    check_app(app, n)
    V = len(cams)
    dev = means.device
    norm = torch.empty((V, n), dtype=torch.float32, device=dev)
    absg = torch.empty((V, n, 2), dtype=torch.float32, device=dev) if opts.absgrad else None
    g = gaussians_struct(*params, app)
    wsz = lib.gs_render_bwd_workspace_size(n * V)
    wbuf = ws.get("bwd", wsz + 256, dev)
    g2 = C.c_void_p(Workspace.aligned(wbuf))
    if seg is None:
        n_tiles, _ = views_extent(cams)
        ssz = lib.gs_seg_workspace_size(n_tiles, int(pair_vals.numel()))
        seg_ptr, seg_bytes, seg_ready = *_seg_args(ws.get("seg", ssz + 256, dev)), 0
    else:
        seg_ptr, seg_bytes, seg_ready = *_seg_args(seg), 1
    cont = lambda t: t.contiguous() if t is not None else None
    d_rgb, d_depth, d_alpha = cont(d_rgb), cont(d_depth), cont(d_alpha)
    cams_c, opt_c, proj_c = L.make_cameras(cams), opts.c(), proj.c()
    _mark("bwd_begin")
    main = torch.cuda.current_stream(dev)
    beside = n >= FILL_BESIDE_MIN
    if beside:
        before = torch.cuda.Event()
        before.record(main)
    L.check(lib.gs_composite_bwd(C.byref(proj_c), _ptr(pair_vals), _ptr(ranges), cams_c, V, C.byref(opt_c), _ptr(T),
                                 _ptr(last), _ptr(d_rgb), _ptr(d_depth), _ptr(d_alpha), int(bool(opts.absgrad)), n * V,
                                 g2, seg_ptr, seg_bytes, seg_ready, _stream()))
    if beside:
        # the gradient arrays are zeroed on a second stream beside the
        # compositing backward (issue-bound, it leaves most of the memory
        # bandwidth free; beside binning or the compositing forward the
        # fill slows them by more than it saves); the projection backward
        # then writes the seen Gaussians' rows only
        grads, zeroed = _zeroed_grads(params, app, before, n)
        _mark("composite_bwd")
        main.wait_event(zeroed)
    else:
        # few Gaussians: the projection backward writes every row itself
        # (the two cross-stream waits would cost more than the fill saves)
        grads = {k: torch.empty_like(t) for k, t in zip(("means", "scales", "quats", "opacities", "sh"), params)}
        if app is not None:
            grads["app"] = torch.empty_like(app)
        _mark("composite_bwd")
    L.check(lib.gs_project_bwd(C.byref(g), cams_c, V, C.byref(opt_c), C.byref(proj_c), g2, C.byref(_grad_struct(grads)),
                               _ptr(norm), _ptr(absg), int(beside), _stream()))
    _mark("project_bwd")
    grads["mean2d_grad_norm"] = norm
    grads["absgrad"] = absg
    grads["_grad2d_ws"] = (wbuf, n * V)
    return grads


def grad2d_view(grads: dict) -> torch.Tensor:
    """The per-slot 2D gradients [S, 12] left in the backward workspace."""
    wbuf, S = grads["_grad2d_ws"]
    off = Workspace.aligned(wbuf) - wbuf.data_ptr()
    return wbuf[off:off + S * 48].view(torch.float32).view(S, 12)


class RenderStats:
    """Filled by the backward: per-view |dL/d mean2d| [V, N] in pixels, and
    (with absgrad) the per-pixel absolute accumulation [V, N, 2]; by the
    forward: n_pairs (an int, or a PairCount whose int() waits for it)."""
    mean2d_grad_norm = None
    absgrad = None
    n_pairs = 0


class GsRasterize(torch.autograd.Function):
    """Differentiable rasterization of several views of the same Gaussians.
    Returns flat per-pixel outputs rgb [Npix, 3], depth [Npix] (sum of
    z * alpha * T) and alpha [Npix]."""

    @staticmethod
    def forward(ctx, means, scales, quats, opacities, sh, app, cams, opts: RenderOptions, stats: RenderStats):
        params = tuple(t.detach().contiguous() for t in (means, scales, quats, opacities, sh))
        app = app.detach().contiguous() if app is not None else None
        n = params[0].shape[-1]
        proj = project(*params, cams, opts, app=app)
        _mark("project")
        # asynchronous once the workspace knows a pair capacity for this
        # size (checked at the end of the backward, or by reading
        # stats.n_pairs)
        known = (n * len(cams), views_extent(cams)[0]) in _default_ws.pair_caps
        pair_vals, ranges, P = bin_sort(proj, cams, n, sync=not known)
        _mark("bin_sort")
        # the forward writes the segment states of the long lists into an
        # area of this call's own, which the backward reads
        seg = seg_workspace(cams, pair_vals)
        out = render_fwd(proj, pair_vals, ranges, cams, opts, seg=seg)
        _mark("render_fwd")
        ctx.save_for_backward(*params, proj.rec, proj.rect, proj.tiles, proj.depth_key, proj.tile_order, pair_vals,
                              ranges, out["T"], out["last"], app)
        ctx.cams, ctx.opts, ctx.stats, ctx.n_pairs, ctx.n_slots = list(cams), opts, stats, P, n * len(cams)
        ctx.seg = seg
        if stats is not None:
            stats.n_pairs = P
        return out["rgb"], out["depth"], out["alpha"]

    @staticmethod
    def backward(ctx, d_rgb, d_depth, d_alpha):
        (means, scales, quats, opacities, sh, rec, rect, tiles, dkey, order, pair_vals, ranges, T,
         last, app) = ctx.saved_tensors
        proj = Projected(rec, rect, tiles, dkey, order)
        g = render_bwd((means, scales, quats, opacities, sh), ctx.cams, ctx.opts, proj, pair_vals, ranges, T, last,
                       d_rgb, d_depth, d_alpha, app=app, seg=ctx.seg)
        ctx.seg = None
        if ctx.stats is not None:
            ctx.stats.mean2d_grad_norm = g["mean2d_grad_norm"]
            ctx.stats.absgrad = g["absgrad"]
        # the forward's binning ran without a read-back; its count is known
        # by now (the whole backward is enqueued behind it)
        P = ctx.n_pairs
        if isinstance(P, PairCount) and P.overflowed():
            _default_ws.pair_caps[(ctx.n_slots, views_extent(ctx.cams)[0])] = _pair_capacity(int(P))
            raise L.GsError(L.GS_ERR_CAPACITY, f"the forward needed {int(P)} pairs but had room for {P.capacity}; "
                                               f"the capacity has been grown, repeat the step")
        return g["means"], g["scales"], g["quats"], g["opacities"], g["sh"], g.get("app"), None, None, None


def rasterize(means, scales, quats, opacities, sh, cams, opts: RenderOptions | None = None,
              stats: RenderStats | None = None, app=None):
    """Autograd entry point; returns flat (rgb, depth, alpha) over all views.
    ``app`` [N, 4]: appearance offsets (dc, do), differentiable."""
    return GsRasterize.apply(means, scales, quats, opacities, sh, app, list(cams), opts or RenderOptions(), stats)


class L1DepthLoss(torch.autograd.Function):
    """Training loss of the library's fused kernel: mean |rgb - target_rgb|
    + lambda * mean |depth / max(alpha, 1e-10) - target_depth| (the depth
    term is dropped when target_depth is None).  The forward computes the
    loss and its gradient in one pass; the backward scales the gradient."""

    @staticmethod
    def forward(ctx, rgb, depth, alpha, target_rgb, target_depth, lambda_depth: float):
        lib = L.load()
        n_pix = rgb.shape[0]
        rgb, target_rgb = rgb.detach().contiguous(), target_rgb.detach().contiguous()
        if rgb.shape != (n_pix, 3) or target_rgb.shape != (n_pix, 3):
            raise ValueError("rgb and target_rgb must be [n_pix, 3]")
        has_d = target_depth is not None
        depth, alpha = depth.detach().contiguous(), alpha.detach().contiguous()
        td = target_depth.detach().contiguous() if has_d else None
        for t in (rgb, target_rgb, depth, alpha) + ((td,) if has_d else ()):
            if not (t.is_cuda and t.dtype == torch.float32):
                raise ValueError("loss inputs must be float32 CUDA tensors")
        if depth.numel() != n_pix or alpha.numel() != n_pix or (has_d and td.numel() != n_pix):
            raise ValueError("depth, alpha and target_depth need one value per pixel")
        loss = torch.empty((1,), dtype=torch.float32, device=rgb.device)
        d_rgb, d_depth, d_alpha = torch.empty_like(rgb), torch.empty_like(depth), torch.empty_like(alpha)
        wsz = lib.gs_loss_workspace_size(n_pix)
        ws = _default_ws.get("loss", wsz + 256, rgb.device)
        L.check(lib.gs_loss_l1_depth(_ptr(rgb), _ptr(depth), _ptr(alpha), _ptr(target_rgb), _ptr(td), n_pix,
                                     float(lambda_depth), _ptr(loss), _ptr(d_rgb), _ptr(d_depth), _ptr(d_alpha),
                                     C.c_void_p(Workspace.aligned(ws)), wsz, _stream()))
        ctx.save_for_backward(d_rgb, d_depth, d_alpha)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        # one multi-tensor launch scales the three gradients
        d_rgb, d_depth, d_alpha = torch._foreach_mul(list(ctx.saved_tensors), g)
        return d_rgb, d_depth, d_alpha, None, None, None


def l1_depth_loss(rgb, depth, alpha, target_rgb, target_depth=None, lambda_depth: float = 0.5):
    return L1DepthLoss.apply(rgb, depth, alpha, target_rgb, target_depth, lambda_depth)


class DSSIMLoss(torch.autograd.Function):
    """weight * (1 - mean SSIM) of one image [H, W, 3] against a target
    (11x11 Gaussian window, sigma 1.5), value and gradient in the library's
    kernels; the backward scales the gradient."""

    @staticmethod
    def forward(ctx, rgb, target, weight: float):
        lib = L.load()
        if rgb.dim() != 3 or rgb.shape[-1] != 3 or tuple(target.shape) != tuple(rgb.shape):
            raise ValueError("rgb and target must be [H, W, 3]")
        rgb, target = rgb.detach().contiguous(), target.detach().contiguous()
        for t in (rgb, target):
            if not (t.is_cuda and t.dtype == torch.float32):
                raise ValueError("D-SSIM inputs must be float32 CUDA tensors")
        H, W = int(rgb.shape[0]), int(rgb.shape[1])
        loss = torch.empty((1,), dtype=torch.float32, device=rgb.device)
        d_rgb = torch.empty_like(rgb)
        wsz = lib.gs_dssim_workspace_size(W, H)
        ws = _default_ws.get("dssim", wsz + 256, rgb.device)
        L.check(lib.gs_dssim(_ptr(rgb), _ptr(target), W, H, float(weight), _ptr(loss), _ptr(d_rgb),
                             C.c_void_p(Workspace.aligned(ws)), wsz, _stream()))
        ctx.save_for_backward(d_rgb)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        (d_rgb,) = ctx.saved_tensors
        return d_rgb * g, None, None


def dssim_loss(rgb, target, weight: float = 0.2):
    return DSSIMLoss.apply(rgb, target, weight)


def split_views(flat: torch.Tensor, cams) -> list:
    """Per-view [H, W, ...] views of a flat per-pixel tensor."""
    sizes = [int(c.width) * int(c.height) for c in cams]
    parts = torch.split(flat, sizes, dim=0)
    return [p.view(int(c.height), int(c.width), *flat.shape[1:]) for p, c in zip(parts, cams)]
