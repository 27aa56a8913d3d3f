"""FP64 CPU oracle of the differentiable tile rasterizer.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, by the smoke check and
by the benchmark's CPU-baseline leg.  The GPU library and its Python
binding never import this package, and this package never imports them.

The arithmetic lives in ``oracle.c`` (double precision, one pixel at a
time); this module compiles it with gcc, marshals NumPy arrays through
ctypes and chains the stages into a forward and a backward.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

TILE = 16
ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4
GUARD_SKIP, GUARD_STOP, GUARD_CLAMP = 1, 2, 4


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_DEFAULT_SOURCE",
                               "-Wall", "-Wno-unknown-pragmas", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Cam(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("R", C.c_double * 9), ("t", C.c_double * 3), ("W", C.c_int32), ("H", C.c_int32),
                ("znear", C.c_double), ("zfar", C.c_double)]


class _Opt(C.Structure):
    _fields_ = [("sh_degree", C.c_int32), ("dilation", C.c_double), ("aa", C.c_int32),
                ("bg", C.c_double * 3)]


_P = C.c_void_p


class _Proj(C.Structure):
    _fields_ = [(name, _P) for name in ("visible", "tcam", "cov2d", "rho", "conic", "mean2d", "depth",
                                        "opac", "rgb", "clamped", "extent", "radius", "rect", "tiles")]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = C.CDLL(_LIB_PATH)
            lib.orc_project.restype = C.c_int
            lib.orc_bin.restype = C.c_int64
            lib.orc_render.restype = C.c_int
            lib.orc_render_bwd.restype = C.c_int
            lib.orc_project_bwd.restype = C.c_int
            lib.orc_num_threads.restype = C.c_int
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def num_threads() -> int:
    return int(_load().orc_num_threads())


def make_cam(cam) -> _Cam:
    vm = np.asarray(cam.viewmat, np.float32).astype(np.float64)
    c = _Cam()
    c.fx, c.fy = float(np.float32(cam.fx)), float(np.float32(cam.fy))
    c.cx, c.cy = float(np.float32(cam.cx)), float(np.float32(cam.cy))
    for i in range(3):
        for j in range(3):
            c.R[3 * i + j] = vm[i, j]
        c.t[i] = vm[i, 3]
    c.W, c.H = int(cam.width), int(cam.height)
    c.znear, c.zfar = float(np.float32(cam.near)), float(np.float32(cam.far))
    return c


def make_opt(sh_degree=3, dilation=0.3, aa=False, bg=(0.0, 0.0, 0.0)) -> _Opt:
    o = _Opt()
    o.sh_degree = int(sh_degree)
    o.dilation = float(np.float32(dilation))
    o.aa = int(bool(aa))
    for k in range(3):
        o.bg[k] = float(np.float32(bg[k]))
    return o


def _c64(a):
    """Parameters enter the oracle as float64 (float32 inputs convert exactly)."""
    return np.ascontiguousarray(a, dtype=np.float64)


def sh_basis(dirs: np.ndarray) -> np.ndarray:
    """Real SH basis (16 functions, degree <= 3) at unit directions [n][3]."""
    d = np.ascontiguousarray(dirs, np.float64)
    out = np.empty((d.shape[0], 16), np.float64)
    _load().orc_sh_basis(C.c_int64(d.shape[0]), _ptr(d), _ptr(out))
    return out


def project(scene, cam, opac=None, cbase=None, **opt) -> dict:
    """Per-Gaussian FP64 projection of one view (EWA, colour, the 3-sigma
    tile rectangle; tile culling belongs to bin_pairs).
    opac replaces the scene's opacities and cbase [n][3] the colour
    constant 1/2 (both for appearance offsets)."""
    lib = _load()
    n = scene.n
    out = {
        "visible": np.zeros(n, np.int32), "tcam": np.zeros((n, 3)), "cov2d": np.zeros((n, 3)),
        "rho": np.zeros(n), "conic": np.zeros((n, 3)), "mean2d": np.zeros((n, 2)), "depth": np.zeros(n),
        "opac": np.zeros(n), "rgb": np.zeros((n, 3)), "clamped": np.zeros((n, 3), np.int32),
        "extent": np.zeros(n), "radius": np.zeros(n, np.int32), "rect": np.zeros((n, 4), np.int32),
        "tiles": np.zeros(n, np.int32),
    }
    pr = _Proj(*[out[k].ctypes.data for k, _ in _Proj._fields_])
    means, scales, quats = _c64(scene.means), _c64(scene.scales), _c64(scene.quats)
    opac, sh = _c64(scene.opacities if opac is None else opac), _c64(scene.sh)
    cb = None if cbase is None else _c64(cbase).reshape(n, 3)
    c, o = make_cam(cam), make_opt(**opt)
    lib.orc_project(C.c_int64(n), _ptr(means), _ptr(scales), _ptr(quats), _ptr(opac), _ptr(sh), _ptr(cb),
                    C.byref(c), C.byref(o), C.byref(pr))
    return out


def depth_key(depth: np.ndarray) -> np.ndarray:
    """Sort key of a view-space depth: the bit pattern of its float32 value
    (monotone for positive depths)."""
    return np.ascontiguousarray(np.asarray(depth, np.float64).astype(np.float32)).view(np.uint32)


def bin_pairs(rect, tiles, depth_keys, slot_view, cams, mask=None, reach=None) -> dict:
    """Pairs (global tile, slot) sorted by (tile, depth key, slot) and the
    [start, end) range of every global tile; views are concatenated.  mask
    [slots] (uint64, optional) selects covered tiles of each rectangle (0:
    all of it), as a compared implementation reports them; reach = (mean2d,
    conic, opac) slot arrays turns on tile culling: a tile is kept only where
    some pixel centre passes the blend's skip rule (oracle.c tile_reached).
    Also returns the pair count of every slot ("tiles")."""
    lib = _load()
    rect = np.ascontiguousarray(rect, np.int32)
    tiles = np.ascontiguousarray(tiles, np.int32)
    mask = np.ascontiguousarray(mask, np.uint64) if mask is not None else None
    depth_keys = np.ascontiguousarray(depth_keys, np.uint32)
    slot_view = np.ascontiguousarray(slot_view, np.int32)
    if reach is not None:
        rm, rc, ro = (np.ascontiguousarray(a, np.float64) for a in reach[:3])
        assert rm.shape == (len(tiles), 2) and rc.shape == (len(tiles), 3) and ro.shape == (len(tiles),)
    else:
        rm = rc = ro = None
    tx = np.array([c.tiles_x for c in cams], np.int32)
    vw = np.array([c.width for c in cams], np.int32)
    vh = np.array([c.height for c in cams], np.int32)
    counts = np.array([c.n_tiles for c in cams], np.int64)
    toff = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int32)
    n_tiles = int(counts.sum())
    cap = int(tiles.astype(np.int64).sum())
    pair_tile = np.zeros(max(cap, 1), np.uint32)
    pair_slot = np.zeros(max(cap, 1), np.uint32)
    ranges = np.zeros((n_tiles, 2), np.uint32)
    slot_tiles = np.zeros(len(tiles), np.int32)
    P = lib.orc_bin(C.c_int64(len(tiles)), _ptr(rect), _ptr(tiles), _ptr(mask), _ptr(rm), _ptr(rc), _ptr(ro),
                    _ptr(depth_keys), _ptr(slot_view), _ptr(tx), _ptr(vw), _ptr(vh), _ptr(toff), C.c_int64(n_tiles),
                    C.c_int64(cap), _ptr(pair_tile), _ptr(pair_slot), _ptr(ranges), _ptr(slot_tiles))
    assert 0 <= P <= cap, (P, cap)
    return {"pair_tile": pair_tile[:P], "pair_slot": pair_slot[:P], "ranges": ranges,
            "tile_off": toff.astype(np.int64), "n_pairs": int(P), "tiles": slot_tiles}


def _twod(proj_list):
    """Concatenate per-view 2D quantities into slot-indexed float64 arrays."""
    cat = lambda k: np.ascontiguousarray(np.concatenate([p[k] for p in proj_list], 0), np.float64)
    return cat("mean2d"), cat("conic"), cat("opac"), cat("rgb"), cat("depth")


# Guard band of a compared float32 implementation (composite_pixel in
# oracle.c), from the unit roundoff u = 2^-24 of its operations:
#   e_0 = 5u      exp (2u), o' (u), o' G' (u), the float32 value of 1/255 (u);
#   e_T = 2u      1 - alpha and T (1 - alpha), one rounding each (and, once
#                 more in the stop test, the float32 value of 1e-4: 0.4u);
#   e_clamp       the float32 clamp 0.99f: 1 - 0.99f is 9.5e-7 off 0.01;
#   e_mean = u    tile-relative mean and dx, each at its own magnitude;
#   e_quad = 5u   float32 conic coefficients (u) and the products and the two
#                 fused sums of the three-term exponent, relative to the terms.
_U = 2.0 ** -24
DEFAULT_GUARD = (5 * _U, 2 * _U, 1e-6, _U, 5 * _U)
STAGE_GUARD = DEFAULT_GUARD


def render_view(cam, opt: dict, tile_off: int, twod, pair_slot, ranges, tile_mask=None,
                guard_eps=DEFAULT_GUARD) -> dict:
    lib = _load()
    mean2d, conic, opac, rgb, depth = twod
    H, W = cam.height, cam.width
    out = {"rgb": np.zeros((H, W, 3)), "depth": np.zeros((H, W)), "alpha": np.zeros((H, W)),
           "T": np.zeros((H, W)), "last": np.zeros((H, W), np.int32), "guard": np.zeros((H, W), np.uint8)}
    g = np.ascontiguousarray(guard_eps, np.float64) if guard_eps is not None else None
    mask = np.ascontiguousarray(tile_mask, np.uint8) if tile_mask is not None else None
    pair_slot = np.ascontiguousarray(pair_slot, np.uint32)
    ranges = np.ascontiguousarray(ranges, np.uint32)
    mean2d, conic, opac, rgb, depth = (np.ascontiguousarray(a, np.float64) for a in (mean2d, conic, opac, rgb, depth))
    lib.orc_render(C.byref(make_cam(cam)), C.byref(make_opt(**opt)), C.c_int64(tile_off), _ptr(mean2d),
                   _ptr(conic), _ptr(opac), _ptr(rgb), _ptr(depth), _ptr(pair_slot),
                   _ptr(ranges), _ptr(mask), _ptr(g), _ptr(out["rgb"]),
                   _ptr(out["depth"]), _ptr(out["alpha"]), _ptr(out["T"]), _ptr(out["last"]), _ptr(out["guard"]))
    return out


def render_alternatives(cam, opt: dict, tile_off: int, twod, pair_slot, ranges, pixels,
                        guard_eps=DEFAULT_GUARD, max_flags: int = 4):
    """For pixels (flat indices y * W + x) of one view: the outputs of the
    blend under every combination of the pixel's flagged decisions taken
    either way (each is a valid result of a float32 evaluation).  Returns
    (alts [n, 2^max_flags, 5] = rgb, depth, alpha; n_alt [n]: 2^m, or -m
    for more than max_flags decisions)."""
    lib = _load()
    pix = np.ascontiguousarray(pixels, np.int64)
    n = len(pix)
    alts = np.full((n, 1 << max_flags, 5), np.nan)
    n_alt = np.zeros(n, np.int32)
    if n == 0:
        return alts, n_alt
    mean2d, conic, opac, rgb, depth = (np.ascontiguousarray(a, np.float64) for a in twod)
    g = np.ascontiguousarray(guard_eps, np.float64)
    pair_slot = np.ascontiguousarray(pair_slot, np.uint32)
    ranges = np.ascontiguousarray(ranges, np.uint32)
    lib.orc_render_alternatives(C.byref(make_cam(cam)), C.byref(make_opt(**opt)), C.c_int64(tile_off),
                                _ptr(mean2d), _ptr(conic), _ptr(opac), _ptr(rgb), _ptr(depth), _ptr(pair_slot),
                                _ptr(ranges), _ptr(g), C.c_int64(n), _ptr(pix), C.c_int(max_flags), _ptr(alts),
                                _ptr(n_alt))
    return alts, n_alt


def compare_image(cam, opt: dict, tile_off: int, twod, pair_slot, ranges, ref: dict, got: dict,
                  tol: float = 1e-4, guard_eps=DEFAULT_GUARD, max_flags: int = 4, where=None) -> dict:
    """Compares a compared implementation's image ``got`` (rgb [H][W][3],
    depth, alpha) with the oracle's ``ref`` (a render_view output over the
    same lists): outside the guard band within tol (rgb, alpha absolute,
    depth relative to max(1, depth)); a flagged pixel must match one of the
    alternatives its flagged decisions allow (render_alternatives).  Returns
    the worst error outside the band and the counts: flagged pixels,
    resolved ones, unresolved ones (more decisions than max_flags) and
    mismatches (flagged pixels matching no alternative).  ``where`` (bool
    [H][W]) limits the comparison to some pixels."""
    has_d, has_a = "depth" in got, "alpha" in got      # rgb alone (a served image) is compared too

    def err(g_rgb, g_d, g_a, r_rgb, r_d, r_a):
        e = np.abs(g_rgb - r_rgb).max(-1)
        if has_a:
            e = np.maximum(e, np.abs(g_a - r_a))
        if has_d:
            e = np.maximum(e, np.abs(g_d - r_d) / np.maximum(1.0, np.abs(r_d)))
        return e
    got = dict(got)
    got.setdefault("depth", ref["depth"])
    got.setdefault("alpha", ref["alpha"])
    e = err(got["rgb"], got["depth"], got["alpha"], ref["rgb"], ref["depth"], ref["alpha"])
    use = np.ones(e.shape, bool) if where is None else np.asarray(where, bool)
    flagged = (ref["guard"] != 0) & use
    worst = float(e[~flagged & use].max(initial=0.0))
    fi = np.flatnonzero(flagged)
    alts, n_alt = render_alternatives(cam, opt, tile_off, twod, pair_slot, ranges, fi, guard_eps, max_flags)
    gr = got["rgb"].reshape(-1, 3)[fi]
    gd, ga = got["depth"].reshape(-1)[fi], got["alpha"].reshape(-1)[fi]
    ea = err(gr[:, None, :], gd[:, None], ga[:, None], alts[..., :3], alts[..., 3], alts[..., 4])
    ok_alt = np.nanmin(np.where(np.isnan(ea), np.inf, ea), axis=1) <= tol
    resolvable = n_alt > 0
    return {"worst": worst, "flagged": int(len(fi)), "resolved": int((resolvable & ok_alt).sum()),
            "unresolved": int((~resolvable).sum()), "mismatch": int((resolvable & ~ok_alt).sum()),
            "mismatch_pixels": fi[resolvable & ~ok_alt][:10].tolist()}


def render_bwd_view(cam, opt: dict, tile_off: int, twod, pair_slot, ranges, g_rgb, g_depth, g_alpha,
                    d2, absg, tile_mask=None):
    lib = _load()
    mean2d, conic, opac, rgb, depth = twod
    g_rgb = np.ascontiguousarray(g_rgb, np.float64)
    g_depth = np.ascontiguousarray(g_depth, np.float64)
    g_alpha = np.ascontiguousarray(g_alpha, np.float64)
    mask = np.ascontiguousarray(tile_mask, np.uint8) if tile_mask is not None else None
    pair_slot = np.ascontiguousarray(pair_slot, np.uint32)
    ranges = np.ascontiguousarray(ranges, np.uint32)
    mean2d, conic, opac, rgb, depth = (np.ascontiguousarray(a, np.float64) for a in (mean2d, conic, opac, rgb, depth))
    assert d2.dtype == np.float64 and d2.flags.c_contiguous
    assert absg is None or (absg.dtype == np.float64 and absg.flags.c_contiguous)
    lib.orc_render_bwd(C.byref(make_cam(cam)), C.byref(make_opt(**opt)), C.c_int64(tile_off), _ptr(mean2d),
                       _ptr(conic), _ptr(opac), _ptr(rgb), _ptr(depth), _ptr(pair_slot), _ptr(ranges),
                       _ptr(mask), _ptr(g_rgb), _ptr(g_depth), _ptr(g_alpha), _ptr(d2), _ptr(absg))


def project_bwd(scene, cam, opt: dict, d2_view, grads: dict, opac=None, cbase=None):
    """Adds one view's parameter gradients into ``grads`` (float64 arrays in
    the parameter layouts; with cbase also grads["cbase"] [n][3]); returns
    |d mean2d| per Gaussian.  ``grads["opacities"]`` is the gradient with
    respect to the opacity used (``opac`` when given)."""
    lib = _load()
    n = scene.n
    norm = np.zeros(n)
    # converted copies are held in locals so they outlive the call
    means, scales, quats = _c64(scene.means), _c64(scene.scales), _c64(scene.quats)
    opac, sh = _c64(scene.opacities if opac is None else opac), _c64(scene.sh)
    cb = None if cbase is None else _c64(cbase).reshape(n, 3)
    d2 = np.ascontiguousarray(d2_view, np.float64)
    keys = ("means", "scales", "quats", "opacities", "sh") + (("cbase",) if cb is not None else ())
    for k in keys:
        assert grads[k].dtype == np.float64 and grads[k].flags.c_contiguous
    c, o = make_cam(cam), make_opt(**opt)
    lib.orc_project_bwd(C.c_int64(n), _ptr(means), _ptr(scales), _ptr(quats), _ptr(opac), _ptr(sh), _ptr(cb),
                        C.byref(c), C.byref(o), _ptr(d2), _ptr(grads["means"]), _ptr(grads["scales"]),
                        _ptr(grads["quats"]), _ptr(grads["opacities"]), _ptr(grads["sh"]),
                        _ptr(grads["cbase"]) if cb is not None else None, _ptr(norm))
    return norm


def forward(scene, cams, opt: dict | None = None, guard_eps=DEFAULT_GUARD, depth_keys=None, app=None,
            tile_cull: bool = False) -> dict:
    """Full FP64 forward over one or more views of the same Gaussians.

    Every Gaussian is listed in every tile of its 3-sigma rectangle (the
    plain definition); ``tile_cull`` drops the tiles where it cannot pass the
    skip rule at any pixel centre (bin_pairs), which leaves every image
    unchanged.  ``app`` [n][4]: appearance offsets (dc, do), applied as in
    oracle.appearance.apply_offsets.  Returns per-view images (rgb, depth,
    alpha, T, last, guard) and the intermediate stages (projections, pairs,
    ranges)."""
    opt = dict(opt or {})
    if not isinstance(cams, (list, tuple)):
        cams = [cams]
    opac = cbase = None
    if app is not None:
        from .appearance import apply_offsets
        opac, cbase = apply_offsets(scene.opacities, app)
    projs = [project(scene, c, opac=opac, cbase=cbase, **opt) for c in cams]
    n = scene.n
    rect = np.concatenate([p["rect"] for p in projs], 0)
    tiles = np.concatenate([p["tiles"] for p in projs], 0)
    keys = depth_key(np.concatenate([p["depth"] for p in projs], 0)) if depth_keys is None else depth_keys
    slot_view = np.repeat(np.arange(len(cams), dtype=np.int32), n)
    twod = _twod(projs)
    bins = bin_pairs(rect, tiles, keys, slot_view, cams, reach=twod[:3] if tile_cull else None)
    images = [render_view(c, opt, int(bins["tile_off"][v]), twod, bins["pair_slot"], bins["ranges"],
                          guard_eps=guard_eps) for v, c in enumerate(cams)]
    return {"proj": projs, "bins": bins, "twod": twod, "images": images, "cams": list(cams), "opt": opt,
            "app": None if app is None else np.asarray(app, np.float64).reshape(n, 4), "opac": opac,
            "cbase": cbase}


def backward(scene, fwd: dict, g_images: list, absgrad: bool = True) -> dict:
    """Analytic FP64 gradients for upstream image gradients
    g_images[v] = (g_rgb [H][W][3], g_depth [H][W], g_alpha [H][W])."""
    n = scene.n
    cams, opt, bins, twod = fwd["cams"], fwd["opt"], fwd["bins"], fwd["twod"]
    V = len(cams)
    d2 = np.zeros((V * n, 10))
    absg = np.zeros((V * n, 2)) if absgrad else None
    for v, c in enumerate(cams):
        gr, gd, ga = g_images[v]
        render_bwd_view(c, opt, int(bins["tile_off"][v]), twod, bins["pair_slot"], bins["ranges"], gr, gd, ga,
                        d2, absg)
    grads = {"means": np.zeros((3, n)), "scales": np.zeros((3, n)), "quats": np.zeros((4, n)),
             "opacities": np.zeros(n), "sh": np.zeros((16, 3, n))}
    app = fwd.get("app")
    if app is not None:
        grads["cbase"] = np.zeros((n, 3))
    norms = np.zeros((V, n))
    for v, c in enumerate(cams):
        norms[v] = project_bwd(scene, c, opt, d2[v * n:(v + 1) * n], grads, opac=fwd.get("opac"),
                               cbase=fwd.get("cbase"))
    if app is not None:
        from .appearance import apply_offsets_bwd
        grads["opacities"], grads["app"] = apply_offsets_bwd(scene.opacities, app, grads["opacities"],
                                                             grads.pop("cbase"))
    grads["mean2d_norm"] = norms
    grads["d2"] = d2
    if absg is not None:
        grads["absgrad"] = absg.reshape(V, n, 2)
    return grads


def cov3d(q, s) -> np.ndarray:
    """Sigma = R(q) diag(s)^2 R(q)^T (Eq. 1) of one Gaussian, 3x3."""
    out = np.zeros(9)
    qq = np.ascontiguousarray(q, np.float64)
    ss = np.ascontiguousarray(s, np.float64)
    _load().orc_cov3d(_ptr(qq), _ptr(ss), _ptr(out))
    return out.reshape(3, 3)
