"""Python binding of the library's level-of-detail selection and serving
runtime (include/gs.h).  Marshalling only: selection runs in the library's
host code, rendering in its kernels, queueing and batching in its worker
threads."""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L
from .rasterizer import RenderOptions, _check_param, gaussians_struct


class LodTable:
    """Partition table of a level-of-detail scene whose levels 1..L share
    one set of parameter arrays.  part_min/part_max (P, 3) world AABBs;
    offsets/counts (L, P) ranges of (level, partition); thresholds[k] the
    largest distance at which level L - k is used; margin (metres) grows
    every AABB for the view test."""

    def __init__(self, part_min, part_max, offsets, counts, thresholds, margin: float):
        self.part_min = np.ascontiguousarray(part_min, np.float32)
        self.part_max = np.ascontiguousarray(part_max, np.float32)
        self.offsets = np.ascontiguousarray(offsets, np.int64)
        self.counts = np.ascontiguousarray(counts, np.int64)
        n_levels, n_parts = self.offsets.shape
        if self.counts.shape != (n_levels, n_parts) or self.part_min.shape != (n_parts, 3) \
                or self.part_max.shape != (n_parts, 3) or len(thresholds) != n_levels:
            raise ValueError("inconsistent level-of-detail table shapes")
        if n_levels > L.GS_MAX_LEVELS:
            raise ValueError(f"at most {L.GS_MAX_LEVELS} levels")
        self.thresholds = tuple(float(t) for t in thresholds)
        self.margin = float(margin)
        t = L.GsLodTable()
        t.n_levels, t.n_parts = n_levels, n_parts
        t.part_min, t.part_max = self.part_min.ctypes.data, self.part_max.ctypes.data
        t.offsets, t.counts = self.offsets.ctypes.data, self.counts.ctypes.data
        for k in range(L.GS_MAX_LEVELS):
            t.thresholds[k] = self.thresholds[k] if k < n_levels else math.inf
        t.margin = self.margin
        self._c = t

    @property
    def n_levels(self) -> int:
        return self.offsets.shape[0]

    @property
    def n_parts(self) -> int:
        return self.offsets.shape[1]

    def c(self) -> L.GsLodTable:
        return self._c


def lod_select(table: LodTable, cam, budget: int):
    """-> (levels int32 [P], 0 = culled or dropped; total selected Gaussians)."""
    lib = L.load()
    level = np.zeros(table.n_parts, np.int32)
    total = C.c_int64()
    cams = L.make_cameras([cam])
    L.check(lib.gs_lod_select(C.byref(table.c()), cams, int(budget), C.c_void_p(level.ctypes.data), C.byref(total)))
    return level, int(total.value)


@dataclass
class ServeConfig:
    max_views_per_batch: int = 8
    n_streams: int = 2
    slot_capacity: int = 24_000_000
    pair_capacity: int = 96_000_000
    pixel_capacity: int = 16_777_216
    queue_capacity: int = 4096
    pipeline_depth: int = 2
    persistent_ctas: int = 0
    pairs_per_gaussian: float = 0.0

    def c(self) -> L.GsServeConfig:
        k = L.GsServeConfig()
        k.max_views_per_batch, k.n_streams = int(self.max_views_per_batch), int(self.n_streams)
        k.slot_capacity, k.pair_capacity = int(self.slot_capacity), int(self.pair_capacity)
        k.pixel_capacity, k.queue_capacity = int(self.pixel_capacity), int(self.queue_capacity)
        k.pipeline_depth, k.persistent_ctas = int(self.pipeline_depth), int(self.persistent_ctas)
        k.pairs_per_gaussian = float(self.pairs_per_gaussian)
        return k


class Server:
    """A running server over device-resident level-of-detail parameters
    (kept referenced here for the server's lifetime)."""

    def __init__(self, params, table: LodTable, opts: RenderOptions, cfg: ServeConfig | None = None,
                 device: int = 0):
        means, scales, quats, opacities, sh = params
        n = means.shape[-1]
        for t, name, shape in ((means, "means", (3, n)), (scales, "scales", (3, n)), (quats, "quats", (4, n)),
                               (opacities, "opacities", (n,)), (sh, "sh", (n, 16, 3))):
            _check_param(t, name, shape)
        self._params = params
        self._table = table
        self.cfg = cfg or ServeConfig()
        self._outs = {}
        lib = L.load()
        g = gaussians_struct(*params)
        srv = C.c_void_p()
        L.check(lib.gs_serve_create(C.byref(g), C.byref(table.c()), C.byref(opts.c()), C.byref(self.cfg.c()),
                                    int(device), C.byref(srv)))
        self._srv = srv

    def now(self) -> float:
        return float(L.load().gs_serve_now(self._srv))

    def submit(self, cam, budget: int, out: torch.Tensor, t_arrival: float | None = None) -> int:
        """Queues one request; `out` is a contiguous float32 device tensor
        [H, W, 3] that receives the image, written after the work queued so
        far on the current stream of its device."""
        if not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
                and tuple(out.shape) == (int(cam.height), int(cam.width), 3)):
            raise ValueError("out must be a contiguous float32 CUDA tensor [H, W, 3]")
        lib = L.load()
        ticket = C.c_uint64()
        t = self.now() if t_arrival is None else float(t_arrival)
        stream = torch.cuda.current_stream(out.device).cuda_stream
        L.check(lib.gs_serve_submit(self._srv, L.make_cameras([cam]), int(budget), C.c_void_p(out.data_ptr()),
                                    C.c_void_p(stream), t, C.byref(ticket)))
        self._outs[ticket.value] = out
        return int(ticket.value)

    def poll(self, max_items: int = 256, timeout_us: int = 0) -> list:
        lib = L.load()
        buf = (L.GsCompletion * max_items)()
        n = C.c_int32()
        L.check(lib.gs_serve_poll(self._srv, buf, int(max_items), int(timeout_us), C.byref(n)))
        out = []
        for i in range(n.value):
            c = buf[i]
            self._outs.pop(int(c.ticket), None)
            out.append({"ticket": int(c.ticket), "status": int(c.status), "batch_views": int(c.batch_views),
                        "n_gaussians": int(c.n_gaussians), "n_pairs": int(c.n_pairs), "t_arrival": c.t_arrival,
                        "t_start": c.t_start, "t_done": c.t_done})
        return out

    def stats(self) -> dict:
        st = L.GsServeStats()
        L.check(L.load().gs_serve_stats_get(self._srv, C.byref(st)))
        return {name: getattr(st, name) for name, _ in L.GsServeStats._fields_}

    def close(self) -> None:
        if self._srv:
            L.check(L.load().gs_serve_destroy(self._srv))
            self._srv = None
            self._outs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
