"""Level-of-detail selection: the oracle (oracle/lod.py) pinned against
brute force, a hand-derived fixture and invariants, then the library's
selection (host code behind gs_lod_select) against the oracle.  CPU only."""
import math
import os

import numpy as np
import pytest

import synthetic as S
from oracle import lod as O

HERE = os.path.dirname(os.path.abspath(__file__))


def cam_at(eye, yaw, pitch, W=640, H=360, hfov=70.0):
    f = W / (2.0 * math.tan(math.radians(hfov) / 2.0))
    d = (math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch))
    target = tuple(e + k for e, k in zip(eye, d))
    return S.Camera(f, f, W / 2.0, H / 2.0, S.look_at(eye, target), W, H)


def random_table(rng, n_parts=24, n_levels=3):
    lo = rng.uniform(-60, 60, (n_parts, 3)).astype(np.float32)
    lo[:, 2] = rng.uniform(-2, 2, n_parts)
    size = rng.uniform(2, 25, (n_parts, 3)).astype(np.float32)
    hi = (lo + size).astype(np.float32)
    base = rng.integers(0, 50, n_parts)
    counts = np.stack([base * (1 + 2 * l) + rng.integers(0, 5, n_parts) for l in range(n_levels)]).astype(np.int64)
    return lo, hi, counts


def in_frustum_points(cam, pts):
    vm = np.asarray(cam.viewmat, np.float64)
    p = pts @ vm[:3, :3].T + vm[:3, 3]
    ulo, uhi, vlo, vhi = O.border_ratios(cam)
    z = p[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u, v = p[:, 0] / z, p[:, 1] / z
    return (z > cam.near) & (u > ulo) & (u < uhi) & (v > vlo) & (v < vhi)


def test_view_test_never_culls_a_box_with_a_point_in_the_frustum():
    rng = np.random.default_rng(0)
    culled = kept = 0
    for trial in range(300):
        cam = cam_at((rng.uniform(-20, 20), rng.uniform(-20, 20), 1.7), rng.uniform(0, 2 * math.pi),
                     rng.uniform(-0.3, 0.2))
        lo = rng.uniform(-80, 80, 3)
        hi = lo + rng.uniform(0.5, 30, 3)
        margin = float(rng.uniform(0, 3))
        g = np.linspace(0, 1, 9)
        a, b, c = np.meshgrid(g, g, g, indexing="ij")
        pts = (lo - margin) + np.stack([a.ravel(), b.ravel(), c.ravel()], 1) * ((hi + margin) - (lo - margin))
        vis = O.in_view(cam, lo, hi, margin)
        if in_frustum_points(cam, pts).any():
            assert vis, trial
        kept += vis
        culled += not vis
    assert culled > 30 and kept > 30


def test_view_test_closed_cases():
    cam = cam_at((0.0, 0.0, 1.7), 0.0, 0.0)            # looking along +x
    assert O.in_view(cam, (5, -1, 0), (6, 1, 3), 0.0)              # straight ahead
    assert not O.in_view(cam, (-30, -5, 0), (-20, 5, 3), 0.0)      # behind the camera
    assert not O.in_view(cam, (10, 40, 0), (12, 42, 3), 0.0)       # far left of the 70 deg field
    assert O.in_view(cam, (10, 40, 0), (12, 42, 3), 40.0)          # ... unless grown by a large margin
    assert O.in_view(cam, (-1, -1, 0), (1, 1, 3), 0.0)             # box around the camera


def test_box_distance_by_sampling():
    rng = np.random.default_rng(1)
    for _ in range(50):
        lo = rng.uniform(-10, 10, 3)
        hi = lo + rng.uniform(0.1, 5, 3)
        c = rng.uniform(-15, 15, 3)
        d = O.box_distance(c, lo, hi)
        g = np.linspace(0, 1, 41)
        a, b, e = np.meshgrid(g, g, g, indexing="ij")
        pts = lo + np.stack([a.ravel(), b.ravel(), e.ravel()], 1) * (hi - lo)
        brute = np.sqrt(((pts - c) ** 2).sum(1)).min()
        assert d <= brute + 1e-12
        assert brute - d <= np.linalg.norm(hi - lo) / 40 + 1e-12
    assert O.box_distance(np.array([0.5, 0.5, 0.5]), (0, 0, 0), (1, 1, 1)) == 0.0


def test_level_thresholds():
    th = (30.0, 60.0, math.inf)
    assert [O.level_for_distance(d, th) for d in (0.0, 30.0, 30.5, 60.0, 61.0, 1e6)] == [3, 3, 2, 2, 1, 1]


def _fixture():
    parts, cases = [], []
    for line in open(os.path.join(HERE, "golden", "lod_budget.txt")):
        t = line.split("#")[0].split()
        if not t:
            continue
        if t[0] == "part":
            v = [float(x) for x in t[1:]]
            parts.append(((v[0], v[2], v[4]), (v[1], v[3], v[5]), v[6:9]))
        else:
            cases.append((int(t[1]), None if t[2] == "error" else ([int(x) for x in t[2:7]], int(t[7]))))
    lo = np.array([p[0] for p in parts], np.float32)
    hi = np.array([p[1] for p in parts], np.float32)
    counts = np.array([p[2] for p in parts], np.int64).T
    return lo, hi, counts, cases


def test_budget_fixture():
    lo, hi, counts, cases = _fixture()
    cam = S.Camera(457.0, 457.0, 320.0, 180.0, S.look_at((0, 0, 1.7), (1, 0, 1.7)), 640, 360)
    for budget, want in cases:
        if want is None:
            with pytest.raises(O.BudgetError):
                O.select(lo, hi, counts, (30.0, 60.0, math.inf), 0.0, cam, budget)
        else:
            lv, tot = O.select(lo, hi, counts, (30.0, 60.0, math.inf), 0.0, cam, budget)
            assert lv.tolist() == want[0] and tot == want[1], budget


def test_budget_ties_go_to_the_lower_id():
    # two mirror-image partitions at the same distance
    cam = S.Camera(457.0, 457.0, 320.0, 180.0, S.look_at((0, 0, 1.7), (1, 0, 1.7)), 640, 360)
    lo = np.array([[20, 2, 0], [20, -6, 0]], np.float32)
    hi = np.array([[24, 6, 3], [24, -2, 3]], np.float32)
    counts = np.array([[5, 5], [20, 20], [40, 40]], np.int64)
    lv, tot = O.select(lo, hi, counts, (30.0, 60.0, math.inf), 0.0, cam, 70)
    assert lv.tolist() == [2, 3] and tot == 60


def test_budget_invariants():
    rng = np.random.default_rng(2)
    for _ in range(30):
        lo, hi, counts = random_table(rng)
        cam = cam_at((rng.uniform(-20, 20), 0.0, 1.7), rng.uniform(0, 2 * math.pi), 0.0)
        th = (20.0, 45.0, math.inf)
        full, total0 = O.select(lo, hi, counts, th, 1.0, cam, 10 ** 12)
        prev = None
        for budget in sorted(rng.integers(0, max(1, total0 + 10), 12)):
            try:
                lv, tot = O.select(lo, hi, counts, th, 1.0, cam, int(budget))
            except O.BudgetError:
                assert prev is None      # only the smallest budgets fail
                continue
            assert tot <= budget and np.all(lv <= full)
            if prev is not None:
                assert np.all(lv >= prev)     # a larger budget never lowers a level
            prev = lv


def _lib_table(gs, lo, hi, counts, th, margin):
    L_, P = counts.shape
    offsets = np.cumsum(np.concatenate([[0], counts.ravel()[:-1]])).reshape(L_, P)
    return gs.LodTable(lo, hi, offsets, counts, th, margin)


def test_library_selection_matches_oracle():
    import paper_2507_23006_amd as gs
    from paper_2507_23006_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        gs.build()
    rng = np.random.default_rng(3)
    lo, hi, counts, cases = _fixture()
    th = (30.0, 60.0, math.inf)
    cam = S.Camera(457.0, 457.0, 320.0, 180.0, S.look_at((0, 0, 1.7), (1, 0, 1.7)), 640, 360)
    t = _lib_table(gs, lo, hi, counts, th, 0.0)
    for budget, want in cases:
        if want is None:
            with pytest.raises(gs.GsError) as ei:
                gs.lod_select(t, cam, budget)
            assert ei.value.code == _lib.GS_ERR_BUDGET
        else:
            lv, tot = gs.lod_select(t, cam, budget)
            assert lv.tolist() == want[0] and tot == want[1]
    n_cmp = 0
    for _ in range(60):
        lo, hi, counts = random_table(rng, n_parts=int(rng.integers(1, 40)))
        th = tuple(float(np.float32(x)) for x in sorted(rng.uniform(5, 80, 2))) + (math.inf,)
        margin = float(np.float32(rng.uniform(0, 4)))
        cam = cam_at((rng.uniform(-30, 30), rng.uniform(-30, 30), 1.7), rng.uniform(0, 2 * math.pi),
                     rng.uniform(-0.3, 0.1), W=int(rng.integers(64, 1920)), H=int(rng.integers(64, 1080)))
        t = _lib_table(gs, lo, hi, counts, th, margin)
        for budget in (10 ** 12, int(rng.integers(0, 2000)), int(rng.integers(0, 200))):
            try:
                want = O.select(lo, hi, counts, th, margin, cam, budget)
            except O.BudgetError:
                with pytest.raises(gs.GsError):
                    gs.lod_select(t, cam, budget)
                continue
            lv, tot = gs.lod_select(t, cam, budget)
            assert lv.tolist() == want[0].tolist() and tot == want[1]
            n_cmp += 1
    assert n_cmp > 100
