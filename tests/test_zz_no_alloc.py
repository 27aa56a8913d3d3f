"""The allocation-free loss entry point (gs_loss_l1_depth_noalloc: its
scratch is a static array of the library) against gs_loss_l1_depth (the
same kernels with a caller workspace), through the C ABI: bitwise equal
loss and gradients on two calls in a row, the second smaller than the
first (the static scratch keeps the first call's partials, which the
second must not read), and the capacity error above 2^26 pixels."""
import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    t = lambda a: torch.from_numpy(a.astype(np.float32)).cuda()
    rgb, trgb = t(rng.random((n, 3))), t(rng.random((n, 3)))
    alpha = t(np.where(rng.random(n) < 0.01, 0.0, rng.uniform(0.05, 1.0, n)))
    depth = t(rng.uniform(1.0, 40.0, n)) * alpha
    tdep = t(rng.uniform(20.0, 45.0, n))
    return rgb, depth, alpha, trgb, tdep


def _call(lib, name, ins, n, lam, ws=None):
    rgb, depth, alpha, trgb, tdep = ins
    p = lambda x: C.c_void_p(x.data_ptr()) if x is not None else None
    out = [torch.full((1,), -1.0, device="cuda"), torch.full_like(rgb, -1.0), torch.full_like(depth, -1.0),
           torch.full_like(alpha, -1.0)]
    args = [p(rgb), p(depth), p(alpha), p(trgb), p(tdep), n, C.c_float(lam)] + [p(o) for o in out]
    if ws is not None:
        args += [C.c_void_p(ws.data_ptr()), ws.numel()]
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(lib, name)(*args, stream)
    torch.cuda.synchronize()
    return rc, out


def test_noalloc_loss_matches_workspace_entry_point(gpu_lib):
    import paper_2507_23006_amd._lib as L
    lib = L.load()
    for n, seed, lam in ((1920 * 1080, 1, 0.5), (160 * 120 + 7, 2, 0.25)):
        ins = _inputs(n, seed)
        ws = torch.empty(lib.gs_loss_workspace_size(n) + 256, dtype=torch.uint8, device="cuda")
        rc_a, ref = _call(lib, "gs_loss_l1_depth", ins, n, lam, ws)
        rc_b, got = _call(lib, "gs_loss_l1_depth_noalloc", ins, n, lam)
        assert rc_a == 0 and rc_b == 0, lib.gs_last_error()
        for a, b in zip(ref, got):
            assert torch.equal(a, b)
        assert float(got[0]) > 0
    # above the static scratch: a host-side error, nothing launched
    rc, _ = _call(lib, "gs_loss_l1_depth_noalloc", _inputs(1, 3), (1 << 26) + 1, 0.5)
    assert rc == L.GS_ERR_CAPACITY
