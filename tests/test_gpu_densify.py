"""Densification bookkeeping and the 3D smoothing filter on the GPU against
the FP64 oracle (oracle/densify.py), on seeded synthetic statistics.

Bars: counts exact and the running sums within 1e-6 relative (float32
accumulation of <= 8 terms); actions bit-exact except Gaussians whose
decision lies within float rounding of its boundary (the oracle's FP64 mean
within 1e-6 of tau_i relative -- the kernel forms the mean in float32 --, or
a score within 1e-6 of the budget's last kept score), which are counted and
must be rare; rates, filtered scales / opacities and their gradients within
1e-6 relative, with view tests within 1e-9 of their boundary set aside.
"""
import numpy as np
import pytest
import torch

import synthetic as S
from oracle import densify as OD

pytestmark = pytest.mark.gpu

f32 = lambda x: float(np.float32(x))


def synthetic_stats(n, V, seed):
    rng = np.random.default_rng(seed)
    tiles = ((rng.random((V, n)) < 0.5) * rng.integers(1, 9, (V, n))).astype(np.int32)
    gn = rng.exponential(3e-4, (V, n)).astype(np.float32)
    ab = rng.exponential(2e-4, (V, n, 2)).astype(np.float32)
    return tiles, gn, ab


@pytest.mark.parametrize("n,V", [(1, 1), (1000, 3), (100_003, 5)])
def test_accumulate_matches_oracle(gpu_lib, n, V):
    D = gpu_lib.densify
    tiles, gn, ab = synthetic_stats(n, V, seed=n + V)
    st = D.DensifyStats(n, "cuda")
    scale = [1.0 + 0.5 * v for v in range(V)]
    t = torch.from_numpy(tiles).cuda()
    D.accumulate(st, t, grad_norm=torch.from_numpy(gn).cuda(), view_scale=scale)
    D.accumulate(st, t, absgrad=torch.from_numpy(ab).cuda())
    ra, rc = OD.accumulate(tiles, grad_norm=gn, view_scale=scale)
    ra, rc = OD.accumulate(tiles, absgrad=ab, accum=ra, count=rc)
    assert np.array_equal(st.count.cpu().numpy(), rc)
    np.testing.assert_allclose(st.accum.cpu().numpy(), ra, rtol=1e-6, atol=1e-12)


def _select_case(gpu_lib, n, seed, budgets, box=(-30.0, 30.0), d_max=60.0):
    D = gpu_lib.densify
    rng = np.random.default_rng(seed)
    acc = rng.exponential(4e-4, n).astype(np.float32)
    cnt = rng.integers(0, 6, n).astype(np.int32)
    means = rng.uniform(-120, 120, (3, n)).astype(np.float32)
    scales = np.exp(rng.normal(-3, 0.8, (3, n))).astype(np.float32)
    opac = rng.uniform(0, 1, n).astype(np.float32)
    st = D.DensifyStats(n, "cuda")
    st.accum.copy_(torch.from_numpy(acc))
    st.count.copy_(torch.from_numpy(cnt))
    dm, ds, do = (torch.from_numpy(a).cuda() for a in (means, scales, opac))
    lo, hi = (box[0],) * 3, (box[1],) * 3
    for budget in budgets:
        p = D.DensifyParams(lo, hi, tau_min=2e-4, eta=4.0, d_max=d_max, prune_opacity=0.01, split_scale=0.1,
                            budget=budget)
        act, counts = D.select(st, dm, ds, do, p)
        act = act.cpu().numpy()
        r = OD.select(acc, cnt, means, scales, opac, lo, hi, f32(2e-4), 4.0, d_max, f32(0.01), f32(0.1), budget)
        guard = np.abs(r["mean"] / r["tau"] - 1.0) < 1e-6
        if 0 < r["k"] < len(r["candidates"]):
            kth = r["score"][r["kept"][-1]]
            guard |= (r["score"] > 0) & (np.abs(r["score"] / kth - 1.0) < 1e-6)
        print(f"select n={n} budget={budget}: {int(guard.sum())} decisions within 1e-6 of their boundary")
        assert guard.sum() <= max(2, n // 10000), guard.sum()
        ok = ~guard
        assert np.array_equal(act[ok], r["action"][ok]), (budget, int((act[ok] != r["action"][ok]).sum()))
        if not guard.any():
            assert counts["candidates"] == len(r["candidates"]) and counts["grown"] == len(r["kept"])
        assert counts["pruned"] == int((opac < f32(0.01)).sum()) and counts["room"] == r["k"]


def test_select_matches_oracle_small(gpu_lib):
    n = 20_011
    _select_case(gpu_lib, n, seed=3, budgets=[0, n - 150, n, n + 1000, 10 * n])


def test_select_full_size(gpu_lib):
    """6M Gaussians (the urban block's count) under a budget that keeps part
    of the candidates: the radix-sorted path at full size."""
    n = 6_000_000
    _select_case(gpu_lib, n, seed=4, budgets=[n + 200_000, 2 * n], box=(-40.0, 40.0), d_max=80.0)


def test_select_edge_cases(gpu_lib):
    D = gpu_lib.densify
    st = D.DensifyStats(1, "cuda")
    z = torch.zeros((3, 1), device="cuda")
    p = D.DensifyParams((0, 0, 0), (1, 1, 1), budget=5)
    act, c = D.select(st, z, z + 0.01, torch.full((1,), 0.5, device="cuda"), p)   # never seen: mean 0
    assert act.item() == D.KEEP and c["candidates"] == 0
    with pytest.raises(gpu_lib.GsError):
        D.select(st, z, z, torch.zeros(1, device="cuda"), D.DensifyParams((0, 0, 0), (1, 1, 1), d_max=0.0))


def test_filter_rate_and_filter_match_oracle(gpu_lib):
    D = gpu_lib.densify
    n = 100_003
    rng = np.random.default_rng(7)
    means = rng.uniform(-3, 3, (3, n)).astype(np.float32)
    cams = []
    for k in range(40):                                        # 3 launches of <= 16 cameras
        eye = (4 * np.cos(k), 4 * np.sin(k), rng.uniform(-1, 1))
        cams.append(S.Camera(120.0 + k, 120.0 + k, 80.0, 60.0, S.look_at(eye, (0, 0, 0), up=(0, 0, 1)), 160, 120))
    dm = torch.from_numpy(means).cuda()
    rate = D.filter3d_rate(dm, cams).cpu().numpy()
    rr = OD.filter_rate(means, cams)
    # the kernel tests x / z against the bounds as products; the oracle
    # divides: view tests within rounding of their boundary are set aside
    ok = OD.filter_rate_margin(means, cams) > 1e-9
    print(f"filter rate: {int((~ok).sum())} of {n} view tests within 1e-9 of a boundary")
    assert (~ok).sum() <= 2
    assert np.array_equal((rate == 0)[ok], (rr == 0)[ok]) and (rr > 0).mean() > 0.5
    np.testing.assert_allclose(rate[ok], rr[ok], rtol=1e-6)
    scales = np.exp(rng.normal(-3, 1, (3, n))).astype(np.float32)
    opac = rng.uniform(0.01, 1, n).astype(np.float32)
    s_t = torch.from_numpy(scales).cuda().requires_grad_(True)
    o_t = torch.from_numpy(opac).cuda().requires_grad_(True)
    r_t = torch.from_numpy(rate).cuda()
    s2, o2 = D.filter3d(s_t, o_t, r_t, 0.45)
    s_f = f32(0.45)                 # the ABI takes s_f as float32
    rs, ro = OD.filter_apply(scales, opac, rate, s_f)
    np.testing.assert_allclose(s2.detach().cpu().numpy(), rs, rtol=1e-6)
    np.testing.assert_allclose(o2.detach().cpu().numpy(), ro, rtol=1e-6, atol=1e-12)
    ws, wo = rng.normal(size=(3, n)).astype(np.float32), rng.normal(size=n).astype(np.float32)
    ((s2 * torch.from_numpy(ws).cuda()).sum() + (o2 * torch.from_numpy(wo).cuda()).sum()).backward()
    rds, rdo = OD.filter_bwd(scales, opac, rate, s_f, ws, wo)
    np.testing.assert_allclose(s_t.grad.cpu().numpy(), rds, rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(o_t.grad.cpu().numpy(), rdo, rtol=1e-6, atol=1e-12)
