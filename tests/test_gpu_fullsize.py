"""Parity at the benchmark's full size and launch configuration: the 6M-Gaussian
urban block at 1920x1080 with anti-aliasing, the same calls bench.py times.
The FP64 oracle renders the whole image (OpenMP over tiles, ~tens of seconds
on the host), so the comparison covers every pixel; gradients are compared
per parameter group over all Gaussians."""
import numpy as np
import pytest
import torch

import oracle
import synthetic as S
from gpu_util import decode_rect, gpu_forward, grads_oracle_layout, oracle_opt, to_dev, view_images

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def c3():
    return S.scene_c3(seed=0), S.camera_c3(seed=2)


def test_c3_forward_and_binning(gpu_lib, c3):
    scene, cam = c3
    cams = [cam]
    opts = gpu_lib.RenderOptions(sh_degree=3, aa=True)
    _, proj, pairs, ranges, P, out = gpu_forward(gpu_lib, scene, cams, opts)
    tiles = proj.tiles.cpu().numpy()
    rect = decode_rect(proj.rect.cpu().numpy(), tiles, cams, scene.n)
    keys = proj.depth_key.cpu().numpy().view(np.uint32)
    f = oracle.forward(scene, cam, oracle_opt(opts), guard_eps=oracle.DEFAULT_GUARD)
    p = f["proj"][0]
    # projection-level integer agreement (rectangles from FP64 on both sides)
    assert np.array_equal(tiles, p["tiles"])
    assert np.array_equal(rect, p["rect"])
    assert np.array_equal(keys[tiles > 0], oracle.depth_key(p["depth"])[tiles > 0])
    # binning: bit-exact against the oracle's own sort of the same keys
    assert P == f["bins"]["n_pairs"]
    assert np.array_equal(pairs.cpu().numpy().view(np.uint32), f["bins"]["pair_slot"])
    assert np.array_equal(ranges.cpu().numpy().view(np.uint32), f["bins"]["ranges"])
    ref = f["images"][0]
    g = {k: view_images(out[k].cpu().numpy(), cams)[0] for k in ("rgb", "depth", "alpha")}
    ok = ref["guard"] == 0
    assert (~ok).sum() <= 1e-3 * cam.n_pixels
    assert np.abs(g["rgb"] - ref["rgb"]).max(-1)[ok].max() <= 1e-4
    assert np.abs(g["alpha"] - ref["alpha"])[ok].max() <= 1e-4
    assert (np.abs(g["depth"] - ref["depth"]) / np.maximum(1.0, ref["depth"]))[ok].max() <= 1e-4


def test_c3_gradients(gpu_lib, c3):
    scene, cam = c3
    opts = gpu_lib.RenderOptions(sh_degree=3, aa=True, absgrad=True)
    w = S.linear_loss_weights(cam.height, cam.width, seed=7)
    params = to_dev(scene, requires_grad=True)
    stats = gpu_lib.RenderStats()
    rgb, depth, alpha = gpu_lib.rasterize(*params, [cam], opts, stats)
    loss = ((torch.from_numpy(w[0]).cuda().view(-1, 3) * rgb).sum() + (torch.from_numpy(w[1]).cuda().view(-1) * depth).sum()
            + (torch.from_numpy(w[2]).cuda().view(-1) * alpha).sum())
    loss.backward()
    torch.cuda.synchronize()
    f = oracle.forward(scene, cam, oracle_opt(opts))
    ref = oracle.backward(scene, f, [w])
    g = grads_oracle_layout(params)
    for k in ("means", "scales", "quats", "opacities", "sh"):
        a = g[k].ravel()
        b = ref[k].ravel()
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        assert rel <= 1e-3, (k, rel)
        rms = np.sqrt(np.mean(b * b))
        good = np.abs(a - b) <= 1e-3 * np.abs(b) + 1e-3 * rms
        assert good.mean() >= 0.999, (k, good.mean())
    rn = ref["mean2d_norm"]
    assert np.linalg.norm(stats.mean2d_grad_norm.cpu().numpy() - rn) / np.linalg.norm(rn) <= 1e-3
