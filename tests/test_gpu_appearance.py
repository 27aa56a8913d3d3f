"""Appearance transform module on the GPU (matrix-core MLP and the offsets'
path through projection) against the FP64 oracle.

Tolerances: the MLP runs in FP32 (matrix-core products with FP32
accumulation over K <= 64 terms of O(1) values, FP32 sigmoid), so offsets
agree to |d| <= 2e-5; gradients per group to a relative norm <= 1e-4 and
elementwise as in the rasterizer's gradient tests.  Renders and gradients
with offsets use the rasterizer's tolerances.
"""
import numpy as np
import pytest
import torch

import oracle
import synthetic as S
from oracle import appearance as OA
from gpu_util import check_image, grads_oracle_layout, oracle_opt, to_dev, view_images

pytestmark = pytest.mark.gpu


def mlp_inputs(n, seed):
    rng = np.random.default_rng(seed)
    g = rng.normal(0, 1, (n, 16)).astype(np.float32)
    g = np.ascontiguousarray(g)
    if n > 5:
        g[3] = 0.0                       # the norm floor
    e = rng.normal(0, 1, 32).astype(np.float32)
    w1 = rng.normal(0, 0.4, (32, 48)).astype(np.float32)
    b1 = rng.normal(0, 0.2, 32).astype(np.float32)
    w2 = rng.normal(0, 0.5, (4, 32)).astype(np.float32)
    b2 = rng.normal(0, 0.2, 4).astype(np.float32)
    return g, e, w1, b1, w2, b2


def gpu_mlp(gs, ins, dy, reg_weight, d_reg):
    t = [torch.from_numpy(a).cuda().requires_grad_(True) for a in ins]
    p = gs.AppearanceParams(*t[2:])
    y, reg = gs.appearance_offsets(t[0], t[1], p, reg_weight)
    (y * torch.from_numpy(dy).cuda()).sum().add(reg * d_reg).backward()
    torch.cuda.synchronize()
    return y.detach().cpu().numpy(), float(reg), [x.grad.cpu().numpy() for x in t]


def compare_group(got, ref, name, rel_tol=1e-4):
    a, b = np.asarray(got, np.float64).ravel(), np.asarray(ref, np.float64).ravel()
    nb = np.linalg.norm(b)
    rel = np.linalg.norm(a - b) / max(nb, 1e-30)
    assert rel <= rel_tol, (name, rel)
    rms = np.sqrt(np.mean(b * b))
    good = np.abs(a - b) <= 1e-3 * np.abs(b) + 1e-3 * rms
    assert good.mean() >= 0.999, (name, good.mean())


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 100_003])
def test_mlp_matches_oracle(gpu_lib, n):
    ins = mlp_inputs(n, seed=n)
    rng = np.random.default_rng(n + 1)
    dy = rng.normal(0, 1, (n, 4)).astype(np.float32)
    y, reg, grads = gpu_mlp(gpu_lib, ins, dy, 0.3, 1.7)
    f = OA.mlp_forward(*ins)
    assert np.abs(y - f["y"]).max() <= 2e-5
    assert abs(reg - OA.opacity_reg(f["y"], 0.3)) <= 1e-6
    ref = OA.mlp_backward(f, dy, 0.3 * 1.7)
    names = ("gemb", "iemb", "w1", "b1", "w2", "b2")
    keep = np.ones(n, bool)
    if n > 5:
        keep[3] = False                  # scaled by 1 / 1e-12: compared relative below
        np.testing.assert_allclose(grads[0][3], ref["gemb"][3], rtol=1e-4, atol=0)
    compare_group(grads[0][keep], ref["gemb"][keep], "gemb")
    for k in range(1, 6):
        compare_group(grads[k], ref[names[k]], names[k])


def test_mlp_empty_input(gpu_lib):
    ins = mlp_inputs(0, seed=0)
    y, reg, grads = gpu_mlp(gpu_lib, ins, np.zeros((0, 4), np.float32), 0.3, 1.0)
    assert y.shape == (0, 4) and reg == 0.0
    for g in grads[1:]:
        assert (g == 0).all()


def test_mlp_full_size_sampled(gpu_lib):
    """6M Gaussians (the urban block's count) in one launch: offsets and
    embedding gradients on 20k sampled rows, weight gradients (sums over
    all 6M) against the oracle's chunked FP64 sums."""
    n = 6_000_000
    ins = mlp_inputs(n, seed=9)
    # Input recipe: embeddings whose FP64 pre-activation lies within 1e-5 of
    # the ReLU kink are re-drawn, so that float32 rounding cannot flip a
    # unit on against the oracle (192M units would otherwise hold a few).
    rng = np.random.default_rng(11)
    for _ in range(20):
        near = np.zeros(n, bool)
        for s in range(0, n, 500_000):
            a = OA.mlp_forward(ins[0][s:s + 500_000], *ins[1:])["a"]
            near[s:s + 500_000] = (np.abs(a) < 1e-5).any(1)
        near[3] = False
        if not near.any():
            break
        ins[0][near] = rng.normal(0, 1, (int(near.sum()), 16)).astype(np.float32)
    assert not near.any()
    rng = np.random.default_rng(10)
    dy = rng.normal(0, 1, (n, 4)).astype(np.float32)
    y, reg, grads = gpu_mlp(gpu_lib, ins, dy, 0.1, 1.0)
    idx = np.sort(rng.choice(n, 20_000, replace=False))
    idx = idx[idx != 3]
    fs = OA.mlp_forward(ins[0][idx], *ins[1:])
    assert np.abs(y[idx] - fs["y"]).max() <= 2e-5
    # the sampled rows' embedding gradients need the regulariser share of the whole set
    fs_dy = dy[idx].astype(np.float64).copy()
    fs_dy[:, 3] += 0.1 / n
    rs = OA.mlp_backward(fs, fs_dy, 0.0)
    compare_group(grads[0][idx], rs["gemb"], "gemb")
    tot = {k: 0.0 for k in ("w1", "b1", "w2", "b2")}
    sum_do = 0.0
    for s in range(0, n, 500_000):
        sl = slice(s, min(n, s + 500_000))
        f = OA.mlp_forward(ins[0][sl], *ins[1:])
        d = dy[sl].astype(np.float64).copy()
        d[:, 3] += 0.1 / n
        r = OA.mlp_backward(f, d, 0.0)
        for k in tot:
            tot[k] = tot[k] + r[k]
        sum_do += f["y"][:, 3].sum()
    assert abs(reg - 0.1 * sum_do / n) <= 1e-6
    for k, gi in (("w1", 2), ("b1", 3), ("w2", 4), ("b2", 5)):
        compare_group(grads[gi], tot[k], k)


def _offsets(n, seed):
    rng = np.random.default_rng(seed)
    return np.column_stack([rng.uniform(0.2, 0.8, (n, 3)), rng.uniform(0.0, 0.6, n)]).astype(np.float32)


def test_identity_offsets_are_bitwise_plain(gpu_lib):
    scene = S.scene_c1()
    cams = [S.camera_c1()]
    opts = gpu_lib.RenderOptions(aa=True)
    params = to_dev(scene)
    plain = [t.cpu().numpy() for t in gpu_lib.rasterize(*params, cams, opts)]
    ident = torch.tensor([0.5, 0.5, 0.5, 0.0], device="cuda").repeat(scene.n, 1).contiguous()
    with_app = [t.cpu().numpy() for t in gpu_lib.rasterize(*params, cams, opts, app=ident)]
    for a, b in zip(plain, with_app):
        assert np.array_equal(a, b)


def test_render_with_offsets_matches_oracle(gpu_lib):
    """Forward images and every gradient (offsets included) of a linear
    functional of the render, with random offsets, against the oracle."""
    scene = S.random_scene(3001, seed=5, log_scale_mu=-2.6)
    cam = S.Camera(120.0, 120.0, 173 / 2.0, 91 / 2.0, S.look_at((1.6, -1.1, -3.3), (0.05, 0.1, 0.0),
                                                                  up=(0.3, -1, 0.2)), 173, 91)
    cams = [cam, S.camera_c1()]
    opts = gpu_lib.RenderOptions(aa=True, bg=(0.1, 0.2, 0.3))
    app_np = _offsets(scene.n, 3)
    params = to_dev(scene, requires_grad=True)
    app = torch.from_numpy(app_np).cuda().requires_grad_(True)
    rgb, depth, alpha = gpu_lib.rasterize(*params, cams, opts, app=app)
    ws = [S.linear_loss_weights(c.height, c.width, seed=7 + v) for v, c in enumerate(cams)]
    cat = lambda i, shape: torch.from_numpy(np.concatenate([w[i].reshape(shape) for w in ws])).cuda()
    loss = (cat(0, (-1, 3)) * rgb).sum() + (cat(1, -1) * depth).sum() + (cat(2, -1) * alpha).sum()
    loss.backward()
    torch.cuda.synchronize()
    f = oracle.forward(scene, cams, oracle_opt(opts), app=app_np)
    for v, c in enumerate(cams):
        got = {"rgb": view_images(rgb.detach().cpu().numpy(), cams)[v],
               "depth": view_images(depth.detach().cpu().numpy(), cams)[v]}
        check_image(c, oracle_opt(opts), int(f["bins"]["tile_off"][v]), f["twod"], f["bins"]["pair_slot"],
                    f["bins"]["ranges"], f["images"][v], got, f"offsets view {v}")
    ref = oracle.backward(scene, f, ws)
    g = grads_oracle_layout(params)
    for k in ("means", "scales", "quats", "opacities", "sh"):
        compare_group(g[k], ref[k], k, rel_tol=1e-3)
    compare_group(app.grad.cpu().numpy(), ref["app"], "app", rel_tol=1e-3)


def test_offsets_chain_through_the_mlp(gpu_lib):
    """gauss_emb -> MLP -> offsets -> render -> linear loss, backward to the
    embeddings and the MLP, against the oracle chain."""
    scene = S.scene_c1()
    cams = [S.camera_c1()]
    opts = gpu_lib.RenderOptions()
    ins = mlp_inputs(scene.n, seed=21)
    t = [torch.from_numpy(a).cuda().requires_grad_(True) for a in ins]
    params = to_dev(scene)
    y, reg = gpu_lib.appearance_offsets(t[0], t[1], gpu_lib.AppearanceParams(*t[2:]), 0.05)
    rgb, depth, alpha = gpu_lib.rasterize(*params, cams, opts, app=y)
    w = S.linear_loss_weights(cams[0].height, cams[0].width, seed=8)
    loss = (torch.from_numpy(w[0].reshape(-1, 3)).cuda() * rgb).sum() + (torch.from_numpy(w[1].reshape(-1)).cuda()
                                                                          * depth).sum() + reg
    loss.backward()
    torch.cuda.synchronize()
    fm = OA.mlp_forward(*ins)
    f = oracle.forward(scene, cams, oracle_opt(opts), app=fm["y"])
    rb = oracle.backward(scene, f, [(w[0], w[1], np.zeros_like(w[2]))])
    r = OA.mlp_backward(fm, rb["app"], 0.05)
    names = ("gemb", "iemb", "w1", "b1", "w2", "b2")
    keep = np.arange(scene.n) != 3
    compare_group(t[0].grad.cpu().numpy()[keep], r["gemb"][keep], "gemb", rel_tol=1e-3)
    for k in range(1, 6):
        compare_group(t[k].grad.cpu().numpy(), r[names[k]], names[k], rel_tol=1e-3)
