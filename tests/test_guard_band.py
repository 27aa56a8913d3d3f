"""Pins of the guard band used by every compositing comparison.

The oracle flags a pixel when one of its skip (alpha vs 1/255), clamp
(o' G' vs 0.99) or stop (T (1 - alpha) vs 1e-4) decisions lies within the
error a float32 evaluation of the blend can make (oracle.c composite_pixel,
oracle.DEFAULT_GUARD, derived from the unit roundoff u = 2^-24 of each
float32 operation).  The claim is checked here without the GPU, against a
float32 model of the blend written in NumPy:

* the records are rounded the way a float32 implementation stores them:
  the 2D mean as an integer plus a float32 fraction, taken relative to its
  16x16 tile's origin; the conic as float32 coefficients of a base-2
  exponent; o' as float32;
* per pixel and list entry: dx, dy, the exponent as c (dy dy) fused into
  b (dx dy), fused into a (dx dx), exp2, o' G', the clamp, the skip test,
  T (1 - alpha) and the stop test, with float32 threshold constants;
* every operation either rounds to float32 (NumPy's own rounding) or is
  carried out in FP64 and then moved by a random, an all-upward or an
  all-downward relative error of one unit roundoff (exp2 two), so the check
  covers any implementation whose operations round within those bounds.

Per pixel the decisions are summarised as (entries composited, entries
clamped, last composited position).  Every pixel whose summary differs
between the float32 model and an FP64 evaluation of the same lists must be
flagged; the FP64 evaluation itself must reproduce the oracle's images.
The flagged set must stay small (a bound that is loose by orders of
magnitude would flag most deep pixels)."""
import math

import numpy as np
import pytest

import oracle
import synthetic as S

U = 2.0 ** -24
LOG2E = 1.0 / math.log(2.0)
A_MIN32, A_MAX32, T_MIN32 = (float(np.float32(v)) for v in (1.0 / 255.0, 0.99, 1e-4))


def _padded_lists(f, cam):
    """Per tile, its depth-ordered slot list padded with -1: [tiles, L]."""
    rg = f["bins"]["ranges"].astype(np.int64)
    ps = f["bins"]["pair_slot"].astype(np.int64)
    lens = rg[:, 1] - rg[:, 0]
    L = int(lens.max())
    out = np.full((cam.n_tiles, L), -1, np.int64)
    for t in range(cam.n_tiles):
        out[t, :lens[t]] = ps[rg[t, 0]:rg[t, 1]]
    return out


def _blend(f, cam, mode, seed=0, unit=U, with_depth=False):
    """Decision summary [H, W, 3] and (rgb, T) of a per-pixel blend of the
    oracle's lists.  mode: "f64" (FP64 with the exact thresholds: the
    oracle's own rules), "f32" (float32 operations), or "rand" / "up" /
    "down" (FP64 operations, each moved by a relative error within its
    bound: ``unit`` per operation, two for exp2, and the threshold constants
    off their values by up to one ``unit``)."""
    rng = np.random.default_rng(seed)
    mean2d, conic, opac, rgb, zdep = f["twod"]
    lists = _padded_lists(f, cam)
    nt, L = lists.shape
    ly, lx = np.divmod(np.arange(256), 16)
    ox = (np.arange(nt) % cam.tiles_x * 16).astype(np.float64)[:, None]
    oy = (np.arange(nt) // cam.tiles_x * 16).astype(np.float64)[:, None]
    inside = ((ox + lx[None, :]) < cam.width) & ((oy + ly[None, :]) < cam.height)
    f32 = mode == "f32"

    def rnd(x, k=1):
        """One operation's rounding (k units for exp2)."""
        if mode == "f64":
            return x
        if f32:
            return np.asarray(x, np.float32).astype(np.float64) if k == 1 else x
        if mode == "up":
            return x * (1.0 + k * unit)
        if mode == "down":
            return x * (1.0 - k * unit)
        return x * (1.0 + k * unit * rng.uniform(-1.0, 1.0, np.shape(x)))

    if mode == "f64":
        op = opac
        a_min, a_max, t_min = 1.0 / 255.0, 0.99, 1e-4
    else:
        qa, qb, qc = (rnd(-LOG2E * c) for c in (0.5 * conic[:, 0], conic[:, 1], 0.5 * conic[:, 2]))
        op = rnd(opac)
        if f32:
            a_min, a_max, t_min = A_MIN32, A_MAX32, T_MIN32
        else:
            a_min, a_max, t_min = (rnd(np.float64(v)) for v in (1.0 / 255.0, 0.99, 1e-4))
    mi = np.floor(mean2d)
    mf = rnd(mean2d - mi)
    T = np.ones((nt, 256))
    C = np.zeros((nt, 256, 3))
    D = np.zeros((nt, 256))
    n_comp = np.zeros((nt, 256), np.int64)
    n_clamp = np.zeros((nt, 256), np.int64)
    last = np.zeros((nt, 256), np.int64)
    done = ~inside
    pxr, pyr = lx[None, :] + 0.5, ly[None, :] + 0.5
    for k in range(L):
        act = np.nonzero((lists[:, k] >= 0) & ~done.all(1))[0]    # tiles with live pixels and an entry k
        if len(act) == 0:
            continue
        s = lists[act, k]
        live = ~done[act]
        if mode == "f64":
            # the oracle's expression, in its order
            dx = (ox[act] + pxr) - mean2d[s, 0][:, None]
            dy = (oy[act] + pyr) - mean2d[s, 1][:, None]
            A, B, Cc = conic[s, 0][:, None], conic[s, 1][:, None], conic[s, 2][:, None]
            p = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy
            G = np.exp(p)
        else:
            mx = rnd((mi[s, 0] - ox[act, 0]) + mf[s, 0])[:, None]
            my = rnd((mi[s, 1] - oy[act, 0]) + mf[s, 1])[:, None]
            dx, dy = rnd(pxr - mx), rnd(pyr - my)
            t1 = rnd(qc[s, None] * rnd(dy * dy))
            t2 = rnd(qb[s, None] * rnd(dx * dy) + t1)
            p = rnd(qa[s, None] * rnd(dx * dx) + t2)
            G = np.exp2(p.astype(np.float32)).astype(np.float64) if f32 else rnd(np.exp2(p), 2)
        raw = rnd(op[s, None] * G)
        alpha = np.minimum(a_max, raw)
        keep = live & ~(p > 0.0) & (alpha >= a_min)
        Ta = T[act]
        Tn = rnd(Ta * rnd(1.0 - alpha))
        stop = keep & (Tn < t_min)
        comp = keep & ~stop
        w = np.where(comp, alpha * Ta, 0.0)
        C[act] += w[..., None] * rgb[s][:, None, :]
        D[act] += w * zdep[s][:, None]
        T[act] = np.where(comp, Tn, Ta)
        n_comp[act] += comp
        n_clamp[act] += comp & (raw >= a_max)
        last[act] = np.where(comp, k + 1, last[act])
        done[act] |= stop

    def img(a):
        tl = a.reshape(cam.tiles_y, cam.tiles_x, 16, 16, *a.shape[2:])
        return tl.swapaxes(1, 2).reshape(cam.tiles_y * 16, cam.tiles_x * 16, *a.shape[2:])[:cam.height, :cam.width]
    summary = np.stack([img(n_comp), img(n_clamp), img(last)], -1)
    if with_depth:
        return summary, img(C), img(T), img(D)
    return summary, img(C), img(T)


def _scene(which):
    if which == "dense_c1":
        return S.scene_c1(), S.camera_c1(), dict(aa=False)
    if which == "oblique_aa":
        sc = S.random_scene(12000, seed=31, log_scale_mu=-2.8)
        sc.opacities[:300] = np.float32(0.995)       # clamped entries
        cam = S.Camera(150.0, 150.0, 96.0, 64.0, S.look_at((1.4, -1.3, -3.1), (0.0, 0.1, 0.0)), 192, 128)
        return sc, cam, dict(aa=True)
    sc = S.random_scene(20000, seed=32, log_scale_mu=-3.3, log_scale_sigma=0.9)
    cam = S.Camera(200.0, 200.0, 120.0, 80.0, S.look_at((0.3, 0.2, -3.6), (0.0, 0.0, 0.0)), 240, 160)
    return sc, cam, dict(aa=False)


@pytest.mark.parametrize("which", ["dense_c1", "oblique_aa", "fine"])
def test_guard_band_covers_float32_decisions(which):
    sc, cam, opt = _scene(which)
    opt = dict(opt, sh_degree=3)
    f = oracle.forward(sc, cam, opt, guard_eps=oracle.DEFAULT_GUARD)
    im = f["images"][0]
    flagged = im["guard"] != 0
    ref, C64, T64 = _blend(f, cam, "f64")
    # the FP64 model follows the oracle's rules exactly
    np.testing.assert_array_equal(ref[..., 2], im["last"])
    np.testing.assert_allclose(C64, im["rgb"] - im["T"][..., None] * np.asarray(opt.get("bg", (0, 0, 0))),
                               atol=1e-12)
    np.testing.assert_allclose(T64, im["T"], rtol=1e-12)
    flipped_any = np.zeros_like(flagged)
    for mode, seed in (("f32", 0), ("rand", 1), ("rand", 2), ("up", 0), ("down", 0)):
        got, _, _ = _blend(f, cam, mode, seed)
        flipped = np.any(got != ref, axis=-1)
        bad = flipped & ~flagged
        assert not bad.any(), (mode, seed, int(bad.sum()), np.argwhere(bad)[:5].tolist())
        flipped_any |= flipped
    n_px = cam.n_pixels
    print(f"{which}: {int(flagged.sum())} of {n_px} pixels flagged ({flagged.mean():.1e}), "
          f"{int(flipped_any.sum())} with a decision moved by some float32 model")
    assert flagged.mean() <= 2e-3


@pytest.mark.parametrize("which", ["dense_c1", "fine"])
def test_guard_band_structure_at_coarser_precision(which):
    """The same model with a unit roundoff of 2^-18 instead of 2^-24 and the
    guard scaled alike (the clamp term becomes 99 units: 1 - 0.99 off by 0.99
    units relative to 0.01).  Decisions now move by the hundred, which makes
    the check sharp: none may escape the flags, and the flagged set stays
    within a few times the moved one.  (Run with the exponent's or the
    mean's term of the bound removed, this check fails.)"""
    unit = 2.0 ** -18
    sc, cam, opt = _scene(which)
    opt = dict(opt, sh_degree=3)
    g = (5 * unit, 2 * unit, 99 * unit, unit, 5 * unit)
    f = oracle.forward(sc, cam, opt, guard_eps=g)
    flagged = f["images"][0]["guard"] != 0
    ref, _, _ = _blend(f, cam, "f64")
    moved = np.zeros_like(flagged)
    for mode, seed in (("rand", 1), ("rand", 2), ("rand", 3), ("up", 0), ("down", 0)):
        got, _, _ = _blend(f, cam, mode, seed, unit=unit)
        flipped = np.any(got != ref, axis=-1)
        bad = flipped & ~flagged
        assert not bad.any(), (mode, seed, int(bad.sum()))
        moved |= flipped
    print(f"{which} at 2^-18: {int(flagged.sum())} flagged, {int(moved.sum())} with a moved decision")
    assert moved.sum() >= 50 and flagged.sum() <= 5 * moved.sum()


@pytest.mark.parametrize("which", ["dense_c1", "fine"])
def test_float32_images_match_the_oracle_or_an_alternative(which):
    """Each float32 model's image matches the oracle within 1e-4 outside
    the guard band, and at every flagged pixel matches one of the results
    its flagged decisions allow (oracle.compare_image, the comparison the
    GPU tests make)."""
    sc, cam, opt = _scene(which)
    opt = dict(opt, sh_degree=3)
    f = oracle.forward(sc, cam, opt, guard_eps=oracle.DEFAULT_GUARD)
    ref = f["images"][0]
    args = (cam, opt, 0, f["twod"], f["bins"]["pair_slot"], f["bins"]["ranges"])
    fi = np.flatnonzero(ref["guard"])
    alts, n_alt = oracle.render_alternatives(*args, fi)
    assert np.all(n_alt >= 2)
    np.testing.assert_array_equal(alts[:, 0, :3], ref["rgb"].reshape(-1, 3)[fi])     # nothing flipped
    np.testing.assert_array_equal(alts[:, 0, 3], ref["depth"].reshape(-1)[fi])
    for mode, seed in (("f32", 0), ("rand", 1), ("up", 0), ("down", 0)):
        _, C, T, D = _blend(f, cam, mode, seed, with_depth=True)
        r = oracle.compare_image(*args, ref, {"rgb": C, "depth": D, "alpha": 1.0 - T})
        assert r["worst"] <= 1e-4 and r["mismatch"] == 0 and r["unresolved"] == 0, (mode, r)


def test_boundary_decisions_resolve_to_their_alternatives():
    """Hand-placed decisions on the boundary: Gaussian 0 reaches alpha
    (1 + 1e-9) / 255 at pixel (10, 8) and Gaussian 3, behind the dense
    Gaussians 1 and 2, takes T to (1 - 1e-9) 1e-4 at pixel (3, 12).  A float32
    model may take either decision the other way; the oracle flags both
    pixels, and the model's result there matches an alternative (the skip
    moves the colour by about 1/255, far beyond the tolerance)."""
    cam = S.Camera(20.0, 20.0, 8.0, 8.0, np.eye(4, dtype=np.float32), 16, 16)
    s2 = 4.0
    p0 = -0.5 * (2.5 ** 2 + 0.5 ** 2) / s2
    flat = [1e-6, 0.0, 1e-6]
    mean2d = np.full((4, 2), 8.0)
    conic = np.array([[1.0 / s2, 0.0, 1.0 / s2], flat, flat, flat])
    # pixel (3, 12): entries 1 and 2 leave T = 0.05 * 0.1, entry 3 takes it to 1e-4 (1 - 1e-9)
    g12 = np.exp(-0.5 * 1e-6 * ((3.5 - 8.0) ** 2 + (12.5 - 8.0) ** 2))
    a3 = 1.0 - 1e-4 * (1.0 - 1e-9) / (0.05 * 0.1)
    opac = np.array([(1.0 + 1e-9) / 255.0 / np.exp(p0), 0.95 / g12, 0.9 / g12, a3 / g12])
    rgb = np.array([[1.0, 1.0, 1.0], [0.2, 0.3, 0.4], [0.1, 0.1, 0.1], [5.0, 5.0, 5.0]])
    depth = np.array([1.0, 2.0, 3.0, 4.0])
    f = {"twod": (mean2d, conic, opac, rgb, depth),
         "bins": {"pair_slot": np.arange(4, dtype=np.uint32), "ranges": np.array([[0, 4]], np.uint32)}}
    opt = dict(sh_degree=0)
    args = (cam, opt, 0, f["twod"], f["bins"]["pair_slot"], f["bins"]["ranges"])
    ref = oracle.render_view(*args)
    assert ref["guard"][8, 10] & oracle.GUARD_SKIP and ref["guard"][12, 3] & oracle.GUARD_STOP
    base = _blend(f, cam, "f64")[0]
    needed = set()
    for mode, seed in (("f32", 0), ("up", 0), ("down", 0), ("rand", 1), ("rand", 2), ("rand", 3)):
        summ, C, T, D = _blend(f, cam, mode, seed, with_depth=True)
        r = oracle.compare_image(*args, ref, {"rgb": C, "depth": D, "alpha": 1.0 - T})
        assert r["worst"] <= 1e-4 and r["mismatch"] == 0 and r["unresolved"] == 0, (mode, r)
        # pixels whose decision moved and whose result only an alternative matches
        moved = np.any(summ != base, axis=-1)
        off = np.abs(C - ref["rgb"]).max(-1) > 1e-4
        needed |= {tuple(p) for p in np.argwhere(moved & off).tolist()}
    assert needed >= {(8, 10), (12, 3)}, needed
