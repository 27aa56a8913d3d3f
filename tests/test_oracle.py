"""Pins of the FP64 oracle against mathematics that does not come from the
oracle itself: library routines, closed forms, worked examples derived by
hand, invariants, brute force and finite differences.  CPU only."""
import dataclasses
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import erf, sph_harm_y

import oracle
import synthetic as S
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_cam(W=48, H=40, f=40.0, tz=4.0):
    vm = np.eye(4, dtype=np.float32)
    vm[2, 3] = tz
    return S.Camera(f, f, W / 2.0, H / 2.0, vm, W, H)


def scene64(scene):
    return S.Scene(*(np.asarray(a, np.float64).copy() for a in
                     (scene.means, scene.scales, scene.quats, scene.opacities, scene.sh)))


# ---------------------------------------------------------------- SH basis

def real_sh_scipy(l, m, theta, phi):
    """Real SH from scipy's complex ones (Condon-Shortley phase included):
    m > 0: sqrt2 Re Y_l^m, m < 0: sqrt2 Im Y_l^|m|, m = 0: Y_l^0."""
    if m == 0:
        return sph_harm_y(l, 0, theta, phi).real
    y = sph_harm_y(l, abs(m), theta, phi)
    return math.sqrt(2.0) * (y.real if m > 0 else y.imag)


def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(11)
    d = rng.standard_normal((200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(d[:, 2])
    phi = np.mod(np.arctan2(d[:, 1], d[:, 0]), 2 * np.pi)
    Y = oracle.sh_basis(d)
    for l in range(4):
        for m in range(-l, l + 1):
            ref = real_sh_scipy(l, m, theta, phi)
            np.testing.assert_allclose(Y[:, l * l + l + m], ref, atol=1e-13, err_msg=f"l={l} m={m}")


def test_sh_basis_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi: exact for the degree-6
    # products of two degree-3 harmonics.
    x, w = np.polynomial.legendre.leggauss(8)
    phis = np.arange(16) * 2 * np.pi / 16
    ct, ph = np.meshgrid(x, phis, indexing="ij")
    wt = np.repeat(w[:, None], 16, 1) * (2 * np.pi / 16)
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    Y = oracle.sh_basis(d)
    gram = (Y * wt.reshape(-1, 1)).T @ Y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-12)


def test_sh_dc_only_colour():
    sc = S.random_scene(32, seed=3)
    cam = small_cam()
    p = oracle.project(sc, cam, sh_degree=0)
    vis = p["visible"] == 1
    y00 = 1.0 / (2.0 * math.sqrt(math.pi))
    raw = y00 * sc.sh[0].astype(np.float64).T + 0.5
    np.testing.assert_allclose(p["rgb"][vis], np.maximum(raw, 0.0)[vis], atol=1e-15)


# ------------------------------------------------------- covariance, projection

def test_cov3d_eigen_structure_matches_scipy_rotation():
    rng = np.random.default_rng(5)
    for _ in range(20):
        q = rng.standard_normal(4)
        s = np.exp(rng.normal(-1, 1, 3))
        Sig = oracle.cov3d(q, s)
        R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()   # scipy: (x, y, z, w)
        for k in range(3):
            np.testing.assert_allclose(Sig @ R[:, k], s[k] ** 2 * R[:, k], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(np.linalg.det(Sig), np.prod(s) ** 2, rtol=1e-10)
        assert np.all(np.linalg.eigvalsh(Sig) > 0)


def _one_gaussian(mu, s, q, o=0.5, dc=(1.0, 1.0, 1.0)):
    sh = np.zeros((16, 3, 1), np.float32)
    sh[0, :, 0] = dc
    return S.Scene(np.asarray(mu, np.float32).reshape(3, 1), np.asarray(s, np.float32).reshape(3, 1),
                   np.asarray(q, np.float32).reshape(4, 1), np.asarray([o], np.float32), sh)


def test_projection_isotropic_on_axis_closed_form():
    cam = small_cam(W=64, H=64, f=50.0, tz=0.0)
    for z, s in [(2.0, 0.05), (5.0, 0.3), (10.0, 1.0)]:
        for q in ([1, 0, 0, 0], [0.3, -0.5, 0.7, 0.1]):
            sc = _one_gaussian([0.0, 0.0, z], [s, s, s], q)
            for aa in (False, True):
                p = oracle.project(sc, cam, sh_degree=0, aa=aa)
                v = (50.0 * np.float64(np.float32(s)) / np.float64(np.float32(z))) ** 2
                np.testing.assert_allclose(p["cov2d"][0], [v, 0.0, v], rtol=1e-12, atol=1e-12)
                dil = float(np.float32(0.3))
                np.testing.assert_allclose(p["conic"][0], [1 / (v + dil), 0.0, 1 / (v + dil)], rtol=1e-12, atol=1e-15)
                np.testing.assert_allclose(p["mean2d"][0], [32.0, 32.0], atol=1e-12)
                expect_rho = (v / (v + dil)) if aa else 1.0      # sqrt of det ratio = v/(v+d)
                np.testing.assert_allclose(p["rho"][0], expect_rho, rtol=1e-12)


def test_projection_matches_finite_difference_jacobian():
    """Inside the frustum clamp, Sigma_2D = J W Sigma W^T J^T with J the
    Jacobian of the perspective map, here taken by central differences."""
    cam = S.camera_c2()
    sc = S.random_scene(64, seed=9, lo=(-5, -5, 0), hi=(5, 5, 3), log_scale_mu=-1.0)
    p = oracle.project(sc, cam, sh_degree=0)
    vm = cam.viewmat.astype(np.float64)
    W_, tw = vm[:3, :3], vm[:3, 3]
    fx, fy, cx, cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))

    def persp(t):
        return np.array([fx * t[0] / t[2] + cx, fy * t[1] / t[2] + cy])

    n_checked = 0
    for i in range(sc.n):
        if not p["visible"][i]:
            continue
        t = W_ @ sc.means[:, i].astype(np.float64) + tw
        h = 1e-5 * t[2]
        Jfd = np.stack([(persp(t + h * e) - persp(t - h * e)) / (2 * h) for e in np.eye(3)], 1)
        Sig = oracle.cov3d(sc.quats[:, i].astype(np.float64), sc.scales[:, i].astype(np.float64))
        ref = Jfd @ W_ @ Sig @ W_.T @ Jfd.T
        got = p["cov2d"][i]
        np.testing.assert_allclose([got[0], got[1], got[2]], [ref[0, 0], ref[0, 1], ref[1, 1]],
                                   rtol=1e-6, atol=1e-9 * abs(ref).max())
        np.testing.assert_allclose(p["mean2d"][i], persp(t), rtol=1e-13)
        np.testing.assert_allclose(p["depth"][i], t[2], rtol=1e-14)
        n_checked += 1
    assert n_checked > 20


def test_extent_and_rect_rule():
    """The 3-sigma rectangle rule of the projection."""
    cam = S.camera_c1()
    sc = S.scene_c1()
    p = oracle.project(sc, cam)
    vis = p["visible"] == 1
    cov = p["cov2d"][vis]
    d = float(np.float32(0.3))
    lam = np.linalg.eigvalsh(np.stack([np.stack([cov[:, 0] + d, cov[:, 1]], 1),
                                       np.stack([cov[:, 1], cov[:, 2] + d], 1)], 1))[:, 1]
    np.testing.assert_allclose(p["extent"][vis], 3 * np.sqrt(lam), rtol=1e-12)
    r = np.ceil(3 * np.sqrt(lam))
    m = p["mean2d"][vis]
    rect = p["rect"][vis]
    np.testing.assert_array_equal(rect[:, 0], np.maximum(0, (np.floor(m[:, 0]) - r) // 16))
    np.testing.assert_array_equal(rect[:, 2], np.minimum(cam.tiles_x - 1, (np.floor(m[:, 0]) + r) // 16))
    np.testing.assert_array_equal(rect[:, 1], np.maximum(0, (np.floor(m[:, 1]) - r) // 16))
    np.testing.assert_array_equal(rect[:, 3], np.minimum(cam.tiles_y - 1, (np.floor(m[:, 1]) + r) // 16))
    np.testing.assert_array_equal(p["tiles"][vis], (rect[:, 2] - rect[:, 0] + 1) * (rect[:, 3] - rect[:, 1] + 1))
    assert np.all(p["tiles"][~vis] == 0)


def _alpha_tiles(p, cam, i, rel=0.0):
    """Tiles holding a pixel centre where Gaussian i reaches alpha >=
    (1 + rel) / 255 (FP64 NumPy brute force over its 3-sigma rectangle)."""
    x0, y0, x1, y1 = p["rect"][i]
    xs = np.arange(x0 * 16, min(cam.width, (x1 + 1) * 16)) + 0.5
    ys = np.arange(y0 * 16, min(cam.height, (y1 + 1) * 16)) + 0.5
    X, Y = np.meshgrid(xs, ys)
    dx, dy = X - p["mean2d"][i, 0], Y - p["mean2d"][i, 1]
    A, B, C = p["conic"][i]
    power = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy
    alpha = np.minimum(0.99, p["opac"][i] * np.exp(power))
    hot = (alpha >= (1.0 + rel) / 255.0) & (power <= 0)
    return set(zip((X[hot] // 16).astype(int).tolist(), (Y[hot] // 16).astype(int).tolist()))


def _cases_for_culling(which):
    if which == "c1":
        return S.scene_c1(), S.camera_c1(), {}
    sc = S.random_scene(1500, seed=21, log_scale_mu=-2.4)
    sc.opacities[:40] = np.float32(0.0035)     # below the skip threshold everywhere
    cam = S.Camera(110.0, 110.0, 70.0, 45.0, S.look_at((1.4, -1.3, -3.1), (0.0, 0.1, 0.0)), 140, 90)
    return sc, cam, dict(aa=True)


@pytest.mark.parametrize("which", ["c1", "oblique_aa"])
def test_tile_culling_is_the_per_pixel_skip_rule(which):
    """Tile-based culling (paper §3.4.2) keeps a (Gaussian, tile) pair
    exactly when some pixel centre of the tile passes the skip rule: the C
    oracle's binning against a NumPy brute force over every pixel of every
    rectangle (decisions within 1e-12 of the threshold may go either way)."""
    sc, cam, opt = _cases_for_culling(which)
    p = oracle.project(sc, cam, **opt)
    keys = oracle.depth_key(p["depth"])
    sv = np.zeros(sc.n, np.int32)
    full = oracle.bin_pairs(p["rect"], p["tiles"], keys, sv, [cam])
    cut = oracle.bin_pairs(p["rect"], p["tiles"], keys, sv, [cam], reach=(p["mean2d"], p["conic"], p["opac"]))
    kept = {}
    tile_of = cut["pair_tile"].astype(np.int64)
    slot_of = cut["pair_slot"].astype(np.int64)
    for s_, t in zip(slot_of.tolist(), tile_of.tolist()):
        kept.setdefault(s_, set()).add((t % cam.tiles_x, t // cam.tiles_x))
    dropped_whole = 0
    for i in np.nonzero(p["visible"])[0]:
        need = _alpha_tiles(p, cam, i, rel=1e-12)
        may = _alpha_tiles(p, cam, i, rel=-1e-12)
        got = kept.get(int(i), set())
        assert need <= got <= may, i
        assert cut["tiles"][i] == len(got)
        dropped_whole += not got
    assert cut["n_pairs"] < full["n_pairs"]
    assert np.array_equal(full["tiles"], p["tiles"])
    # the kept pairs are a sub-list of the unculled ones, in the same order
    pos = {(t, s_): k for k, (t, s_) in enumerate(zip(full["pair_tile"].tolist(), full["pair_slot"].tolist()))}
    at = np.array([pos[(t, s_)] for t, s_ in zip(tile_of.tolist(), slot_of.tolist())])
    assert np.all(np.diff(at) > 0)
    if which == "oblique_aa":
        assert dropped_whole >= 40


@pytest.mark.parametrize("aa", [False, True])
def test_tile_culling_leaves_images_unchanged(aa):
    sc = S.random_scene(2500, seed=22, log_scale_mu=-2.5)
    cams = [S.camera_c1(), S.Camera(90.0, 90.0, 50.0, 35.0, S.look_at((1.0, 1.5, -3.0), (0.0, 0.0, 0.0)), 100, 70)]
    opt = dict(aa=aa, bg=(0.1, 0.2, 0.3))
    f0 = oracle.forward(sc, cams, opt, guard_eps=None)
    f1 = oracle.forward(sc, cams, opt, guard_eps=None, tile_cull=True)
    assert f1["bins"]["n_pairs"] < 0.8 * f0["bins"]["n_pairs"]
    for a, b in zip(f0["images"], f1["images"]):
        for k in ("rgb", "depth", "alpha", "T"):
            assert np.array_equal(a[k], b[k]), k


def test_near_plane_culls():
    cam = small_cam(tz=0.0)
    sc = _one_gaussian([0.0, 0.0, 0.005], [0.1] * 3, [1, 0, 0, 0])
    assert oracle.project(sc, cam)["visible"][0] == 0
    sc = _one_gaussian([0.0, 0.0, -1.0], [0.1] * 3, [1, 0, 0, 0])
    assert oracle.project(sc, cam)["visible"][0] == 0


# ------------------------------------------------------------ binning and sort

def test_bin_matches_lexsort_enumeration():
    cams = [S.camera_c1(), dataclasses.replace(small_cam(W=70, H=50, f=45.0))]
    sc = S.random_scene(800, seed=4, log_scale_mu=-2.0)
    projs = [oracle.project(sc, c) for c in cams]
    rect = np.concatenate([p["rect"] for p in projs])
    tiles = np.concatenate([p["tiles"] for p in projs])
    # covered-tile masks as a compared implementation reports them (random
    # subsets of rectangles of <= 64 tiles; 0 = the whole rectangle)
    rng = np.random.default_rng(4)
    area = tiles.astype(np.int64)
    mask = np.zeros(len(tiles), np.uint64)
    for s_ in np.nonzero((area > 1) & (area <= 64))[0]:
        bits = rng.random(area[s_]) < 0.6
        bits[rng.integers(area[s_])] = True
        mask[s_] = np.uint64(sum(1 << int(k) for k in np.nonzero(bits)[0]))
        tiles[s_] = int(bits.sum())
    assert (mask != 0).sum() > 50
    keys = oracle.depth_key(np.concatenate([p["depth"] for p in projs]))
    # force some exact depth ties so the index tie-break is exercised
    keys[10:20] = keys[10]
    slot_view = np.repeat(np.arange(2, dtype=np.int32), sc.n)
    b = oracle.bin_pairs(rect, tiles, keys, slot_view, cams, mask=mask)
    toff = [0, cams[0].n_tiles]
    rows = []
    for s_ in range(len(tiles)):
        if tiles[s_] == 0:
            continue
        v = slot_view[s_]
        x0, y0, x1, y1 = (int(v) for v in rect[s_])
        m = int(mask[s_])
        for ty in range(y0, y1 + 1):
            for tx in range(x0, x1 + 1):
                if m and not (m >> ((ty - y0) * (x1 - x0 + 1) + (tx - x0))) & 1:
                    continue
                rows.append((toff[v] + ty * cams[v].tiles_x + tx, keys[s_], s_))
    rows = np.array(rows, np.int64)
    order = np.lexsort((rows[:, 2], rows[:, 1], rows[:, 0]))
    np.testing.assert_array_equal(b["pair_tile"], rows[order, 0])
    np.testing.assert_array_equal(b["pair_slot"], rows[order, 2])
    # ranges tile [0, P) exactly once
    r = b["ranges"].astype(np.int64)
    nz = r[:, 1] > r[:, 0]
    assert (r[nz, 1] - r[nz, 0]).sum() == b["n_pairs"]
    for t in np.nonzero(nz)[0][:50]:
        assert np.all(b["pair_tile"][r[t, 0]:r[t, 1]] == t)


# ------------------------------------------------------------ compositing rules

def render_2d(cam, opac, rgb, depth, mean2d=None, conic=None, opt=None, guard_eps=oracle.DEFAULT_GUARD):
    """Composites hand-made 2D Gaussians that cover the whole image."""
    n = len(opac)
    mean2d = np.zeros((n, 2)) if mean2d is None else np.asarray(mean2d, np.float64)
    conic = np.zeros((n, 3)) if conic is None else np.asarray(conic, np.float64)
    rect = np.tile(np.array([0, 0, cam.tiles_x - 1, cam.tiles_y - 1], np.int32), (n, 1))
    tiles = np.full(n, cam.n_tiles, np.int32)
    keys = oracle.depth_key(depth)
    b = oracle.bin_pairs(rect, tiles, keys, np.zeros(n, np.int32), [cam])
    twod = (np.ascontiguousarray(mean2d), np.ascontiguousarray(conic), np.asarray(opac, np.float64),
            np.ascontiguousarray(rgb, np.float64), np.asarray(depth, np.float64))
    return oracle.render_view(cam, opt or {}, 0, twod, b["pair_slot"], b["ranges"], guard_eps=guard_eps)


def load_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *v = line.split()
            vals[k] = [float(x) for x in v]
    return vals


def test_alpha_stack_worked_example():
    g = load_golden("alpha_stack.txt")
    n = int(g["n"][0])
    cam = small_cam(W=20, H=18)
    im = render_2d(cam, [g["opacity"][0]] * n, [g["colour"]] * n, g["depths"])
    assert np.all(im["last"] == int(g["last"][0]))
    np.testing.assert_allclose(im["T"], g["T_final"][0], rtol=1e-12)
    np.testing.assert_allclose(im["alpha"], g["alpha"][0], rtol=1e-12)
    np.testing.assert_allclose(im["rgb"], np.broadcast_to(g["rgb"], im["rgb"].shape), rtol=1e-12)
    np.testing.assert_allclose(im["depth"], g["depth"][0], rtol=1e-12)


def test_skip_rule_threshold():
    cam = small_cam(W=16, H=16)
    under = render_2d(cam, [0.003], [[1.0, 1.0, 1.0]], [2.0])
    assert np.all(under["T"] == 1.0) and np.all(under["rgb"] == 0.0) and np.all(under["last"] == 0)
    over = render_2d(cam, [0.005], [[1.0, 1.0, 1.0]], [2.0])
    np.testing.assert_allclose(over["rgb"], 0.005, rtol=1e-14)
    np.testing.assert_allclose(over["depth"], 0.01, rtol=1e-14)
    assert np.all(over["last"] == 1)


def test_alpha_clamp_at_099():
    cam = small_cam(W=16, H=16)
    im = render_2d(cam, [1.0], [[1.0, 0.5, 0.25]], [3.0])
    np.testing.assert_allclose(im["alpha"], 0.99, rtol=1e-14)
    np.testing.assert_allclose(im["rgb"][..., 1], 0.5 * 0.99, rtol=1e-14)


def test_background_term():
    cam = small_cam(W=16, H=16)
    im = render_2d(cam, [0.5], [[0.2, 0.2, 0.2]], [3.0], opt={"bg": (1.0, 0.0, 0.25)})
    np.testing.assert_allclose(im["rgb"][0, 0], [0.1 + 0.5, 0.1, 0.1 + 0.125], rtol=1e-12)


def test_single_gaussian_pixels_and_integral():
    """One isotropic Gaussian: every pixel is c * min(.99, o G'), zero where
    o G' < 1/255; the summed opacity equals o 2 pi sqrt(det Sigma') times
    the mass inside the skip contour, 1 - 1/(255 o) (the mass of a 2D
    Gaussian outside its level set G = g is exactly g)."""
    cam = small_cam(W=128, H=128, f=100.0, tz=0.0)
    o, s, z = 0.5, 0.2, 4.0
    sc = _one_gaussian([0.0, 0.0, z], [s, s, s], [1, 0, 0, 0], o=o, dc=(1.0, 1.0, 1.0))
    f = oracle.forward(sc, cam, {"sh_degree": 0})
    im = f["images"][0]
    p = f["proj"][0]
    ys, xs = np.mgrid[0:128, 0:128] + 0.5
    A, B, Cc = p["conic"][0]
    dx, dy = xs - p["mean2d"][0, 0], ys - p["mean2d"][0, 1]
    G = np.exp(-0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy)
    al = np.minimum(0.99, o * G)
    al[al < 1 / 255] = 0.0
    c = 1.0 / (2 * math.sqrt(math.pi)) + 0.5
    np.testing.assert_allclose(im["rgb"][..., 0], c * al, atol=1e-15)
    np.testing.assert_allclose(im["depth"], float(np.float32(z)) * al, rtol=1e-12, atol=1e-15)
    sigma2 = 1.0 / A
    total = o * 2 * math.pi * sigma2 * (1 - 1 / (255 * o))
    assert p["extent"][0] < 3.2 * math.sqrt(sigma2) + 1 and im["alpha"].sum() == pytest.approx(total, rel=1e-2)
    # erf form of the mass inside the 3-sigma square, as a cross-check of the rectangle
    assert erf(3 / math.sqrt(2)) ** 2 > 0.99


def test_permutation_invariance_bitwise():
    cam = small_cam(W=64, H=48, f=50.0)
    sc = S.random_scene(300, seed=21, log_scale_mu=-2.0)
    base = oracle.forward(sc, cam)["images"][0]
    perm = np.random.default_rng(1).permutation(sc.n)
    pim = oracle.forward(sc.subset(perm), cam)["images"][0]
    for k in ("rgb", "depth", "alpha", "T", "last"):
        assert np.array_equal(base[k], pim[k]), k


def test_depth_ties_follow_index_order():
    cam = small_cam(W=16, H=16)
    # same depth: the lower index is composited first
    im = render_2d(cam, [0.5, 0.5], [[1.0, 0, 0], [0, 1.0, 0]], [2.0, 2.0])
    np.testing.assert_allclose(im["rgb"][0, 0], [0.5, 0.25, 0.0], rtol=1e-14)
    im = render_2d(cam, [0.5, 0.5], [[0, 1.0, 0], [1.0, 0, 0]], [2.0, 2.0])
    np.testing.assert_allclose(im["rgb"][0, 0], [0.25, 0.5, 0.0], rtol=1e-14)


def test_transmittance_bounds_c1():
    f = oracle.forward(S.scene_c1(), S.camera_c1())
    im = f["images"][0]
    assert im["T"].min() >= 1e-4 and im["T"].max() <= 1.0
    assert im["rgb"].min() >= 0.0 and im["depth"].min() >= 0.0
    np.testing.assert_allclose(im["alpha"], 1.0 - im["T"], atol=0)
    assert im["last"].max() > 10


@pytest.mark.parametrize("seed,aa,deg,bg", [(0, False, 3, (0, 0, 0)), (1, True, 3, (0.3, 0.1, 0.9)),
                                            (2, True, 1, (0, 0, 0)), (3, False, 0, (1, 1, 1))])
def test_matches_numpy_brute_force(seed, aa, deg, bg):
    sc = S.random_scene(96, seed=seed, log_scale_mu=-2.3)
    cam = small_cam(W=40 + seed, H=33, f=35.0) if seed % 2 == 0 else oblique_cam(W=40 + seed, H=33, f=35.0)
    opt = dict(sh_degree=deg, aa=aa, bg=bg)
    ref = brute.render(sc, cam, **opt)
    # the brute force lists every Gaussian of the 3-sigma rectangle, so list
    # positions (last) compare with tile culling off; images with it on too
    for cull in (False, True):
        im = oracle.forward(sc, cam, opt, tile_cull=cull)["images"][0]
        for k in ("rgb", "depth", "alpha", "T"):
            np.testing.assert_allclose(im[k], ref[k], atol=1e-13, err_msg=k)
        if not cull:
            np.testing.assert_array_equal(im["last"], ref["last"])


# --------------------------------------------------------------- gradients

def oblique_cam(W=56, H=44, f=45.0):
    """A camera whose rotation is far from the identity (so R and R^T differ)."""
    return S.Camera(f, f, W / 2.0, H / 2.0, S.look_at((1.6, -1.1, -3.3), (0.05, 0.1, 0.0), up=(0.3, -1, 0.2)), W, H)


def _fd_setup(seed=8, n=160, aa=True, bg=(0.2, 0.4, 0.1)):
    sc = scene64(S.random_scene(n, seed=seed, log_scale_mu=-2.0))
    cam = oblique_cam()
    opt = dict(sh_degree=3, aa=aa, bg=bg)
    w = S.linear_loss_weights(cam.height, cam.width, seed=7)
    return sc, cam, opt, w


def _loss(sc, cam, opt, w):
    im = oracle.forward(sc, cam, opt)["images"][0]
    return float((w[0] * im["rgb"]).sum() + (w[1] * im["depth"]).sum() + (w[2] * im["alpha"]).sum())


GROUPS = {"means": (3,), "scales": (3,), "quats": (4,), "opacities": (), "sh": (16, 3)}


def _perturbed(sc, group, idx, delta):
    arrs = {k: getattr(sc, k).copy() for k in GROUPS}
    arrs[group][idx] += delta
    return S.Scene(arrs["means"], arrs["scales"], arrs["quats"], arrs["opacities"], arrs["sh"])


@pytest.mark.parametrize("aa", [False, True])
def test_analytic_gradient_matches_central_differences(aa):
    sc, cam, opt, w = _fd_setup(aa=aa)
    f = oracle.forward(sc, cam, opt)
    g = oracle.backward(sc, f, [w])
    rng = np.random.default_rng(7)
    vis = np.nonzero(f["proj"][0]["tiles"] > 0)[0]
    checked = 0
    for group, shape in GROUPS.items():
        grad = g[group]
        for _ in range(12):
            i = int(rng.choice(vis))
            comp = tuple(int(rng.integers(0, s)) for s in shape)
            idx = comp + (i,)
            theta = getattr(sc, group)[idx]
            h = 1e-6 * max(1.0, abs(theta))
            fd = [(_loss(_perturbed(sc, group, idx, k * h), cam, opt, w) -
                   _loss(_perturbed(sc, group, idx, -k * h), cam, opt, w)) / (2 * k * h) for k in (1, 2)]
            if abs(fd[0] - fd[1]) > 1e-4 * (abs(fd[0]) + 1e-6):
                continue          # a discrete event (skip/stop/rect) lies within 2h: resample
            an = grad[idx]
            assert abs(an - fd[0]) <= 2e-6 * abs(an) + 2e-7, (group, idx, an, fd)
            checked += 1
    assert checked >= 50


def test_mean2d_grad_norm_and_absgrad():
    sc, cam, opt, w = _fd_setup()
    f = oracle.forward(sc, cam, opt)
    g = oracle.backward(sc, f, [w])
    d2 = g["d2"]
    np.testing.assert_allclose(g["mean2d_norm"][0], np.hypot(d2[:, 0], d2[:, 1]), rtol=1e-14)
    ab = g["absgrad"][0]
    assert np.all(ab[:, 0] >= np.abs(d2[:, 0]) - 1e-12) and np.all(ab[:, 1] >= np.abs(d2[:, 1]) - 1e-12)


def test_multi_view_gradients_are_sums_of_single_views():
    sc, cam, opt, _ = _fd_setup(n=120)
    cam2 = S.Camera(cam.fx, cam.fy, cam.cx, cam.cy, S.look_at((0.5, -0.4, -3.5), (0, 0, 0), up=(0, -1, 0)),
                    cam.width, cam.height)
    ws = [S.linear_loss_weights(c.height, c.width, seed=s) for c, s in ((cam, 7), (cam2, 8))]
    fm = oracle.forward(sc, [cam, cam2], opt)
    gm = oracle.backward(sc, fm, ws)
    for v, c in enumerate((cam, cam2)):
        fs = oracle.forward(sc, c, opt)
        for k in ("rgb", "depth", "alpha", "last"):
            np.testing.assert_allclose(fm["images"][v][k], fs["images"][0][k], atol=1e-15)
    g1 = oracle.backward(sc, oracle.forward(sc, cam, opt), [ws[0]])
    g2 = oracle.backward(sc, oracle.forward(sc, cam2, opt), [ws[1]])
    for k in GROUPS:
        np.testing.assert_allclose(gm[k], g1[k] + g2[k], rtol=1e-12, atol=1e-14)


def test_stop_ends_the_pixel():
    """After the entry that would take T below 1e-4, nothing more is
    composited, not even a faint entry that would keep T above 1e-4."""
    cam = small_cam(W=16, H=16)
    op = [0.95, 0.95, 0.95, 0.95, 0.01]
    im = render_2d(cam, op, [[1.0, 1.0, 1.0]] * 5, [1.0, 2.0, 3.0, 4.0, 5.0])
    assert np.all(im["last"] == 3)
    np.testing.assert_allclose(im["T"], 0.05 ** 3, rtol=1e-12)


def test_gradient_with_clamped_jacobian():
    """Gaussians whose mean lies beyond the frustum clamp (15% outside the
    image) but whose footprint reaches into it: the clamped Jacobian's
    gradient still matches central differences."""
    cam = small_cam(W=48, H=40, f=40.0)
    rng = np.random.default_rng(3)
    n = 24
    # means at |u| ~ 0.8-1.1 (the clamp sits at (24 + 7.2) / 40 = 0.78), large scales
    u = rng.uniform(0.85, 1.1, n) * rng.choice([-1, 1], n)
    z = rng.uniform(3.0, 5.0, n)
    means = np.stack([u * (z - 0.0) , rng.uniform(-0.3, 0.3, n), z - 4.0], 0)
    sc = S.random_scene(n, seed=4)
    sc = S.Scene(means.astype(np.float64), np.full((3, n), 0.6), sc.quats.astype(np.float64),
                 sc.opacities.astype(np.float64), sc.sh.astype(np.float64))
    opt = dict(sh_degree=1, aa=True)
    f = oracle.forward(sc, cam, opt)
    p = f["proj"][0]
    umax = (24 + 0.15 * 48) / 40.0
    clamped = (p["tiles"] > 0) & (np.abs(p["tcam"][:, 0] / p["tcam"][:, 2]) > umax)
    assert clamped.sum() >= 5
    w = S.linear_loss_weights(cam.height, cam.width, seed=7)
    g = oracle.backward(sc, f, [w])
    checked = 0
    for i in np.nonzero(clamped)[0]:
        for group, idx in (("means", (0, i)), ("means", (2, i)), ("scales", (0, i)), ("quats", (1, i))):
            theta = getattr(sc, group)[idx]
            h = 1e-6 * max(1.0, abs(theta))
            fd = [(_loss(_perturbed(sc, group, idx, k * h), cam, opt, w) -
                   _loss(_perturbed(sc, group, idx, -k * h), cam, opt, w)) / (2 * k * h) for k in (1, 2)]
            if abs(fd[0] - fd[1]) > 1e-4 * (abs(fd[0]) + 1e-6):
                continue
            assert abs(g[group][idx] - fd[0]) <= 2e-6 * abs(g[group][idx]) + 2e-7, (group, idx, g[group][idx], fd)
            checked += 1
    assert checked >= 12


def test_float32_and_float64_inputs_give_identical_results():
    """The wrapper converts float32 parameters to float64 copies; the copies
    must stay alive through the C calls (a freed copy gives garbage)."""
    sc32 = S.random_scene(300, seed=31, log_scale_mu=-2.0)
    sc64 = scene64(sc32)
    cam = oblique_cam()
    w = S.linear_loss_weights(cam.height, cam.width, seed=7)
    res = []
    for sc in (sc32, sc64):
        f = oracle.forward(sc, cam, dict(aa=True))
        g = oracle.backward(sc, f, [w])
        res.append((f["images"][0]["rgb"], g))
    assert np.array_equal(res[0][0], res[1][0])
    for k in GROUPS:      # the OpenMP backward sums in varying order: equal up to rounding
        np.testing.assert_allclose(res[0][1][k], res[1][1][k], rtol=1e-10, atol=1e-14, err_msg=k)


# --------------------------------------------------------------- loss

def test_loss_fixture_by_hand():
    from oracle import loss as OL
    # one pixel: |(0.5, 0.2, 0.9) - 0.4| = (0.1, 0.2, 0.5) -> 0.8 / 3; expected depth 2 / 0.5 = 4 vs 3 -> 0.5 * 1
    L, dr, dd, da = OL.l1_depth([[0.5, 0.2, 0.9]], [2.0], [0.5], [[0.4, 0.4, 0.4]], [3.0], 0.5)
    assert abs(L - (0.8 / 3 + 0.5)) < 1e-15
    np.testing.assert_allclose(dr, [[1 / 3, -1 / 3, 1 / 3]], rtol=1e-15)
    np.testing.assert_allclose(dd, [0.5 / 0.5], rtol=1e-15)           # lambda * sign / alpha
    np.testing.assert_allclose(da, [-0.5 * 2.0 / 0.25], rtol=1e-15)   # -lambda * sign * D / alpha^2
    # alpha below the clamp: expected depth D / 1e-10, no gradient to alpha
    L, dr, dd, da = OL.l1_depth([[0.0, 0.0, 0.0]], [1e-12], [0.0], [[0.0, 0.0, 0.0]], [0.0], 0.5)
    assert abs(L - 0.5 * 1e-2) < 1e-15 and da[0] == 0.0 and abs(dd[0] - 0.5 / 1e-10) < 1e-3


def test_loss_gradient_by_finite_differences():
    from oracle import loss as OL
    rng = np.random.default_rng(4)
    n = 50
    rgb, t_rgb = rng.random((n, 3)), rng.random((n, 3))
    D, a, td = rng.uniform(1, 5, n), rng.uniform(0.2, 1, n), rng.uniform(1, 20, n)
    L0, dr, dd, da = OL.l1_depth(rgb, D, a, t_rgb, td, 0.7)
    h = 1e-7
    for arr, grad in ((rgb, dr), (D, dd), (a, da)):
        for _ in range(10):
            i = tuple(int(rng.integers(0, s)) for s in arr.shape)
            old = arr[i]
            arr[i] = old + h
            lp = OL.l1_depth(rgb, D, a, t_rgb, td, 0.7)[0]
            arr[i] = old - h
            lm = OL.l1_depth(rgb, D, a, t_rgb, td, 0.7)[0]
            arr[i] = old
            assert abs((lp - lm) / (2 * h) - grad[i]) <= 1e-6 * max(1.0, abs(grad[i]))


# --------------------------------------------------------------- D-SSIM

def test_ssim_window_and_identity():
    from oracle import ssim as OS
    w = OS.window()
    assert len(w) == 11 and abs(w.sum() - 1.0) < 1e-15 and np.allclose(w, w[::-1])
    assert abs(w[6] / w[5] - np.exp(-1.0 / (2 * 1.5 ** 2))) < 1e-14      # Gaussian, sigma 1.5
    x = np.random.default_rng(0).random((20, 17, 3))
    loss, g = OS.dssim(x, x, 0.2)
    assert abs(loss) < 1e-12 and np.abs(g).max() < 1e-12                  # SSIM(x, x) = 1 is a maximum


def test_ssim_of_constant_images_closed_form():
    from oracle import ssim as OS
    a, b = 0.3, 0.7
    s, _ = OS.ssim_map(np.full((31, 31, 3), a), np.full((31, 31, 3), b))
    # away from the border the window sees only constants: zero variances
    want = (2 * a * b + OS.C1) / (a * a + b * b + OS.C1)      # the C2 factors cancel
    np.testing.assert_allclose(s[10:21, 10:21], want, rtol=1e-12)


def test_dssim_gradient_by_finite_differences():
    from oracle import ssim as OS
    rng = np.random.default_rng(1)
    x, y = rng.random((13, 12, 3)), rng.random((13, 12, 3))
    L0, g = OS.dssim(x, y, 0.2)
    h = 1e-6
    for _ in range(25):
        i = tuple(int(rng.integers(0, s)) for s in x.shape)
        old = x[i]
        x[i] = old + h
        lp = OS.dssim(x, y, 0.2)[0]
        x[i] = old - h
        lm = OS.dssim(x, y, 0.2)[0]
        x[i] = old
        assert abs((lp - lm) / (2 * h) - g[i]) <= 1e-7 + 1e-5 * abs(g[i]), i


# --------------------------------------------------------------- appearance transform

def _mlp_inputs(rng, n):
    from oracle import appearance as OA
    return (rng.normal(0, 1, (n, OA.GAUSS_DIM)), rng.normal(0, 1, OA.IMAGE_DIM),
            rng.normal(0, 0.4, (OA.HIDDEN, OA.GAUSS_DIM + OA.IMAGE_DIM)), rng.normal(0, 0.2, OA.HIDDEN),
            rng.normal(0, 0.5, (OA.OUT, OA.HIDDEN)), rng.normal(0, 0.2, OA.OUT))


def test_appearance_mlp_worked_example():
    """A hand-built MLP: g = (3, 4, 0...) normalises to (0.6, 0.8, 0...),
    the image embedding 2 e_31 to e_31; hidden unit 0 sees 0.6 + 0.8 = 1.4,
    unit 1 sees -2 + 0.5 < 0 and is cut by the ReLU; output 3 gets
    ln(3) / 1.4 * 1.4 = ln 3, so its sigmoid is 3/4; the others are sigmoid(0)."""
    from oracle import appearance as OA
    g = np.zeros((1, 16)); g[0, 0], g[0, 1] = 3.0, 4.0
    e = np.zeros(32); e[31] = 2.0
    w1 = np.zeros((32, 48)); w1[0, 0] = w1[0, 1] = 1.0; w1[1, 47] = -2.0
    b1 = np.zeros(32); b1[1] = 0.5
    w2 = np.zeros((4, 32)); w2[3, 0] = math.log(3.0) / 1.4; w2[2, 1] = 100.0
    f = OA.mlp_forward(g, e, w1, b1, w2, np.zeros(4))
    np.testing.assert_allclose(f["y"][0], [0.5, 0.5, 0.5, 0.75], rtol=0, atol=1e-15)
    assert f["h"][0, 1] == 0.0


def test_appearance_mlp_gradient_by_finite_differences():
    from oracle import appearance as OA
    rng = np.random.default_rng(11)
    ins = list(_mlp_inputs(rng, 7))
    dy = rng.normal(0, 1, (7, 4))
    lam = 0.3

    def loss(args):
        f = OA.mlp_forward(*args)
        return float((f["y"] * dy).sum()) + OA.opacity_reg(f["y"], lam), f

    L0, f0 = loss(ins)
    assert np.abs(f0["a"]).min() > 1e-3          # no ReLU kink within the step
    g = OA.mlp_backward(f0, dy, lam)
    names = ("gemb", "iemb", "w1", "b1", "w2", "b2")
    h = 1e-6
    for k, name in enumerate(names):
        arr = ins[k]
        for _ in range(6):
            i = tuple(int(rng.integers(0, s)) for s in arr.shape)
            old = arr[i]
            arr[i] = old + h
            lp = loss(ins)[0]
            arr[i] = old - h
            lm = loss(ins)[0]
            arr[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name][i]) <= 1e-7 + 1e-6 * abs(fd), (name, i, fd, g[name][i])


def test_appearance_mlp_scale_invariance_of_normalised_embeddings():
    """The MLP sees only directions of both embeddings: outputs are invariant
    under positive scaling and each embedding gradient is orthogonal to it."""
    from oracle import appearance as OA
    rng = np.random.default_rng(12)
    gemb, iemb, w1, b1, w2, b2 = _mlp_inputs(rng, 9)
    f = OA.mlp_forward(gemb, iemb, w1, b1, w2, b2)
    scale = rng.uniform(0.1, 10.0, (9, 1))
    f2 = OA.mlp_forward(gemb * scale, iemb * 3.7, w1, b1, w2, b2)
    np.testing.assert_allclose(f2["y"], f["y"], rtol=1e-13, atol=0)
    g = OA.mlp_backward(f, rng.normal(0, 1, (9, 4)), 0.0)
    np.testing.assert_allclose((g["gemb"] * gemb).sum(1), 0.0, atol=1e-13)
    assert abs(float(g["iemb"] @ iemb)) < 1e-12
    # a zero embedding stays finite (the 1e-12 floor of the norm)
    f3 = OA.mlp_forward(np.zeros((1, 16)), iemb, w1, b1, w2, b2)
    assert np.isfinite(f3["y"]).all()


def test_appearance_identity_offsets_leave_the_render_unchanged():
    """dc = 1/2, do = 0 is the identity of the offset rule; do = 1 makes
    every Gaussian transparent."""
    sc, cam = S.random_scene(512, 0), S.camera_c1()
    opt = {"sh_degree": 3}
    base = oracle.forward(sc, cam, opt)["images"][0]
    ident = np.tile([0.5, 0.5, 0.5, 0.0], (sc.n, 1))
    im = oracle.forward(sc, cam, opt, app=ident)["images"][0]
    for k in ("rgb", "depth", "alpha", "T", "last"):
        assert np.array_equal(im[k], base[k]), k
    clear = np.tile([0.5, 0.5, 0.5, 1.0], (sc.n, 1))
    im = oracle.forward(sc, cam, opt, app=clear)["images"][0]
    assert (im["T"] == 1.0).all() and (im["rgb"] == 0.0).all()


def test_appearance_offset_gradients_by_finite_differences():
    """Render gradients with respect to the offsets (through o (1 - do) and
    the colour constant) against FP64 central differences."""
    sc, cam = S.random_scene(256, 3), S.camera_c1()
    opt = {"sh_degree": 3, "aa": True}
    rng = np.random.default_rng(5)
    app = np.column_stack([rng.uniform(0.2, 0.8, (sc.n, 3)), rng.uniform(0.0, 0.5, sc.n)])
    f = oracle.forward(sc, cam, opt, app=app)
    H, W = cam.height, cam.width
    w = (rng.normal(0, 1, (H, W, 3)), rng.normal(0, 1, (H, W)), rng.normal(0, 1, (H, W)))
    g = oracle.backward(sc, f, [w])

    def lin(a):
        im = oracle.forward(sc, cam, opt, app=a)["images"][0]
        return float((im["rgb"] * w[0]).sum() + (im["depth"] * w[1]).sum() + (im["alpha"] * w[2]).sum()), im

    seen = np.nonzero(f["proj"][0]["tiles"] > 0)[0]
    h = 1e-7
    checked = 0
    for i in rng.permutation(seen)[:12]:
        for c in range(4):
            a = app.copy(); a[i, c] += h
            lp, ip = lin(a)
            a[i, c] -= 2 * h
            lm, im_ = lin(a)
            if not (np.array_equal(ip["last"], im_["last"]) and np.array_equal(ip["last"], f["images"][0]["last"])):
                continue                     # the skip/stop set moved inside the step
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g["app"][i, c]) <= 1e-5 * max(1.0, abs(fd)), (i, c, fd, g["app"][i, c])
            checked += 1
    assert checked >= 30
    # the opacity gradient is chained through o (1 - do)
    f0 = oracle.forward(sc, cam, opt, app=None)
    assert np.isfinite(g["opacities"]).all() and f0["app"] is None


# --------------------------------------------------------------- densification bookkeeping

def test_densify_accumulate_worked_example():
    """Two views, three Gaussians: Gaussian 1 unseen in view 0; AbsGS mode
    takes the length of the per-axis sums (3-4-5)."""
    from oracle import densify as OD
    tiles = np.array([[2, 0, 1], [1, 1, 0]])
    gn = np.array([[0.5, 9.0, 1.0], [0.25, 2.0, 7.0]])
    acc, cnt = OD.accumulate(tiles, grad_norm=gn, view_scale=[2.0, 4.0])
    np.testing.assert_array_equal(cnt, [2, 1, 1])
    np.testing.assert_allclose(acc, [0.5 * 2 + 0.25 * 4, 2.0 * 4, 1.0 * 2], rtol=0, atol=0)
    ab = np.zeros((2, 3, 2)); ab[0, 0] = (3.0, 4.0); ab[1, 0] = (6.0, 8.0)
    acc2, cnt2 = OD.accumulate(tiles, absgrad=ab, accum=acc, count=cnt)
    assert acc2[0] == acc[0] + 5.0 + 10.0 and cnt2[0] == 4


def test_densify_threshold_eq4_worked_example():
    """tau_min inside the partition, eta tau_min beyond d_max, linear between:
    d = 30 of d_max = 60 with eta = 4 gives tau_min (0.5 * 3 + 1)."""
    from oracle import densify as OD
    means = np.array([[5.0, 40.0, 200.0, 10.0], [5.0, 5.0, 5.0, -20.0], [0.0, 0.0, 0.0, 40.0]])
    tau, d = OD.thresholds(means, (0.0, 0.0, -100.0), (10.0, 10.0, 100.0), 2e-4, 4.0, 60.0)
    np.testing.assert_allclose(d, [0.0, 30.0, 190.0, 20.0], rtol=1e-15)
    np.testing.assert_allclose(tau, [2e-4, 2.5 * 2e-4, 4 * 2e-4, 2e-4 * (20 / 60 * 3 + 1)], rtol=1e-15)


def test_densify_box_distance_by_dense_sampling():
    from oracle import densify as OD
    rng = np.random.default_rng(3)
    lo, hi = np.array([-2.0, 1.0, 0.0]), np.array([3.0, 2.0, 5.0])
    g = [np.linspace(lo[k], hi[k], 41) for k in range(3)]
    box = np.stack(np.meshgrid(*g, indexing="ij"), -1).reshape(-1, 3)
    pts = rng.uniform(-8, 10, (40, 3))
    d = OD.box_distance(pts.T, lo, hi)
    brute = np.sqrt(((pts[:, None, :] - box[None, :, :]) ** 2).sum(-1)).min(1)
    assert np.all(d <= brute + 1e-12) and np.all(brute - d <= 0.2)   # grid step 0.125 at most


def test_densify_select_worked_example():
    """Six Gaussians, budget for 2 new ones after pruning one: the two
    largest mean / tau win; the larger-scaled of them is split."""
    from oracle import densify as OD
    means = np.zeros((3, 6)); means[0, 5] = 70.0          # Gaussian 5 is 60 m outside: tau = 4 tau_min
    acc = np.array([3.0, 6.0, 1.0, 9.0, 5.0, 12.0]) * 1e-4
    cnt = np.array([1, 2, 1, 3, 1, 1])                    # means 3, 3, 1, 3, 5, 12 (x 1e-4)
    scales = np.full((3, 6), 0.01); scales[1, 4] = 0.5
    opac = np.array([0.5, 0.5, 0.5, 0.001, 0.5, 0.5])      # Gaussian 3 is pruned
    r = OD.select(acc, cnt, means, scales, opac, (-10, -10, -10), (10, 10, 10), 2e-4, 4.0, 60.0, 0.005, 0.1,
                  budget=7)
    # candidates: 0 (1.5), 1 (1.5), 4 (2.5), 5 (12 / 8 = 1.5); 2 is below tau; K = 7 - 5 = 2
    assert r["k"] == 2
    assert list(r["candidates"]) == [0, 1, 4, 5]
    assert list(r["action"]) == [OD.CLONE, OD.KEEP, OD.KEEP, OD.PRUNE, OD.SPLIT, OD.KEEP]


def test_densify_select_invariants():
    from oracle import densify as OD
    rng = np.random.default_rng(4)
    n = 3000
    means = rng.uniform(-50, 50, (3, n))
    acc = rng.exponential(4e-4, n)
    cnt = rng.integers(0, 5, n)
    scales = rng.uniform(0.001, 0.2, (3, n))
    opac = rng.uniform(0, 1, n)
    for budget in (0, n - 50, n + 100, 10 * n):
        r = OD.select(acc, cnt, means, scales, opac, (-10, -10, -5), (10, 10, 5), 2e-4, 4.0, 40.0, 0.01, 0.1, budget)
        a = r["action"]
        assert ((a == OD.PRUNE) == (opac < 0.01)).all()
        kept = np.isin(a, (OD.CLONE, OD.SPLIT))
        assert kept.sum() == min(r["k"], len(r["candidates"]))
        cand = np.zeros(n, bool); cand[r["candidates"]] = True
        assert not (kept & ~cand).any()
        if kept.any() and (cand & ~kept).any():
            assert r["score"][kept].min() >= r["score"][cand & ~kept].max()
        assert ((a == OD.SPLIT) == (kept & (scales.max(0) > 0.1))).all()


def test_filter3d_is_an_isotropic_covariance_addition():
    """R diag(s'^2) R^T = R diag(s^2) R^T + sigma^2 I, and the opacity factor
    is sqrt(det Sigma / det Sigma') (numpy determinants)."""
    from oracle import densify as OD
    rng = np.random.default_rng(5)
    for _ in range(10):
        q = rng.normal(size=4); s = rng.uniform(0.01, 0.5, 3); rate = rng.uniform(50, 500)
        s2, o2 = OD.filter_apply(s[:, None], np.array([0.8]), np.array([rate]), 0.45)
        sig2 = (0.45 / rate) ** 2
        S0 = oracle.cov3d(q, s)
        S1 = oracle.cov3d(q, s2[:, 0])
        np.testing.assert_allclose(S1, S0 + sig2 * np.eye(3), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(o2[0], 0.8 * np.sqrt(np.linalg.det(S0) / np.linalg.det(S1)), rtol=1e-10)
    s2, o2 = OD.filter_apply(np.full((3, 1), 0.1), np.array([0.7]), np.array([0.0]), 0.45)
    assert s2[0, 0] == 0.1 and o2[0] == 0.7                   # unseen: no filter


def test_filter3d_gradient_by_finite_differences():
    from oracle import densify as OD
    rng = np.random.default_rng(6)
    n = 20
    s, o, r = rng.uniform(0.01, 0.3, (3, n)), rng.uniform(0.1, 1, n), rng.uniform(20, 300, n)
    r[3] = 0.0
    ws, wo = rng.normal(size=(3, n)), rng.normal(size=n)
    f = lambda s_, o_: float((OD.filter_apply(s_, o_, r, 0.45)[0] * ws).sum() + (OD.filter_apply(s_, o_, r, 0.45)[1] * wo).sum())
    ds, do = OD.filter_bwd(s, o, r, 0.45, ws, wo)
    h = 1e-7
    for k in range(3):
        for i in range(n):
            sp, sm = s.copy(), s.copy(); sp[k, i] += h; sm[k, i] -= h
            assert abs((f(sp, o) - f(sm, o)) / (2 * h) - ds[k, i]) <= 1e-6 * max(1, abs(ds[k, i]))
    for i in range(n):
        op, om = o.copy(), o.copy(); op[i] += h; om[i] -= h
        assert abs((f(s, op) - f(s, om)) / (2 * h) - do[i]) <= 1e-7


def test_filter3d_rate_closed_forms():
    """On the optical axis at depth z the rate is f / z; behind the camera or
    outside the widened image it is 0; with two cameras the larger wins."""
    from oracle import densify as OD
    cam = S.camera_c1()                                       # f = 150, centre at z = -4 looking +z
    means = np.array([[0.0, 0.0, 0.0, 0.0, 5.0], [0.0, 0.0, 0.0, 0.0, 0.0], [0.0, 2.0, -6.0, 1.0, 0.0]])
    r = OD.filter_rate(means, [cam])
    np.testing.assert_allclose(r[:4], [150 / 4.0, 150 / 6.0, 0.0, 150 / 5.0], rtol=1e-12)
    assert r[4] == 0.0                                        # x / z = 5 / 4 beyond (80 + 24) / 150
    vm = np.array(cam.viewmat, np.float32).copy(); vm[2, 3] = 2.0
    near = S.Camera(cam.fx, cam.fy, cam.cx, cam.cy, vm, cam.width, cam.height)
    r2 = OD.filter_rate(means, [cam, near])
    np.testing.assert_allclose(r2[:2], [150 / 2.0, 150 / 4.0], rtol=1e-12)
