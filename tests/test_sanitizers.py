"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU: the FP64 oracle (gcc) on a small scene through projection, binning
with tile culling, compositing, its alternatives and the backward; and the
library's host code (hipcc, sanitizers on the host pass only) through
level-of-detail selection, argument validation of the C ABI and the
server's create/destroy paths, which fail cleanly without a GPU.  Each run
is a child process with the sanitizer runtime preloaded; any report ends
it with a nonzero status."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1", "OMP_NUM_THREADS": "2"}


def _run(script: str, preload: str, timeout: int = 600) -> str:
    env = dict(os.environ, **SAN_ENV, LD_PRELOAD=preload, PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", textwrap.dedent(script)], env=env, capture_output=True, text=True,
                       timeout=timeout, cwd=ROOT)
    assert r.returncode == 0 and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, \
        r.stdout[-2000:] + r.stderr[-8000:]
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    asan = subprocess.check_output([gcc, "-print-file-name=libasan.so"], text=True).strip()
    ubsan = subprocess.check_output([gcc, "-print-file-name=libubsan.so"], text=True).strip()
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run([gcc, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_DEFAULT_SOURCE",
                    "-o", lib, os.path.join(ROOT, "oracle", "oracle.c"), "-lm"], check=True)
    out = _run(f"""
        import numpy as np
        import oracle
        oracle._LIB_PATH = {lib!r}
        import synthetic as S
        scene = S.random_scene(300, seed=5)
        cams = [S.Camera(40.0, 40.0, 24.0, 17.0, S.look_at((0.2, -0.1, -3.0), (0.0, 0.0, 0.0)), 45, 35),
                S.Camera(30.0, 30.0, 16.0, 16.0, S.look_at((0.5, 0.3, -2.5), (0.0, 0.0, 0.0)), 32, 31)]
        opt = dict(sh_degree=3, dilation=0.3, aa=True, bg=(0.1, 0.2, 0.3))
        f = oracle.forward(scene, cams, opt, guard_eps=oracle.DEFAULT_GUARD, tile_cull=True)
        w = []
        for v, im in enumerate(f["images"]):
            rng = np.random.default_rng(v)
            w.append((rng.standard_normal(im["rgb"].shape), rng.standard_normal(im["depth"].shape),
                      rng.standard_normal(im["alpha"].shape)))
        g = oracle.backward(scene, f, w, absgrad=True)
        assert all(np.isfinite(v).all() for v in g.values() if isinstance(v, np.ndarray))
        r = oracle.compare_image(cams[0], opt, 0, f["twod"], f["bins"]["pair_slot"], f["bins"]["ranges"],
                                 f["images"][0], {{"rgb": f["images"][0]["rgb"]}}, guard_eps=oracle.DEFAULT_GUARD)
        print("ok", f["bins"]["n_pairs"], r["unresolved"])
    """, f"{asan}:{ubsan}")
    assert out.startswith("ok"), out


def _clang_asan_runtime():
    base = "/opt/rocm/llvm/lib/clang"
    if not os.path.isdir(base):
        return None
    for v in sorted(os.listdir(base), reverse=True):
        p = os.path.join(base, v, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    return None


def test_library_host_code_under_asan_ubsan(tmp_path):
    import concurrent.futures as cf
    import importlib
    B = importlib.import_module("paper_2507_23006_amd.build")
    rt = _clang_asan_runtime()
    if rt is None:
        pytest.skip("no clang AddressSanitizer runtime")
    san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"):
        san += ["-Xarch_host", f]
    flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1", "-g"] + san

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        r = subprocess.run([B._hipcc(), *flags, "-x", "hip", "-c", os.path.join(B.CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        return obj

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(compile_one, B.SOURCES))
    lib = str(tmp_path / "libgs_san.so")
    r = subprocess.run([B._hipcc(), "-shared", "-fPIC", f"--offload-arch={B.ARCH}", *san, "-o", lib, *objs],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    out = _run(f"""
        import ctypes as C, math
        import numpy as np
        from paper_2507_23006_amd import _lib as L
        L.LIB_PATH = {lib!r}
        import paper_2507_23006_amd as gs
        import synthetic as S
        lib = L.load()
        # level-of-detail selection, with budgets that drop levels and partitions
        rng = np.random.default_rng(2)
        P, Lv = 30, 3
        lo = rng.uniform(-60, 60, (P, 3)).astype(np.float32)
        hi = (lo + rng.uniform(2, 25, (P, 3))).astype(np.float32)
        base = rng.integers(0, 50, P)
        counts = np.stack([base * (1 + 2 * l) + rng.integers(0, 5, P) for l in range(Lv)]).astype(np.int64)
        offsets = np.cumsum(counts.ravel()).reshape(Lv, P) - counts
        table = gs.LodTable(lo, hi, offsets, counts, (12.0, 30.0, math.inf), 1.5)
        n_sel = 0
        for k in range(40):
            yaw = rng.uniform(0, 2 * math.pi)
            eye = (rng.uniform(-50, 50), rng.uniform(-50, 50), 1.7)
            f = 320.0
            cam = S.Camera(f, f, 320.0, 180.0, S.look_at(eye, (eye[0] + math.cos(yaw), eye[1] + math.sin(yaw), 1.7)),
                           640, 360)
            for budget in (10 ** 9, 400, 50):
                try:
                    lv, tot = gs.lod_select(table, cam, budget)
                    n_sel += tot
                except L.GsError as e:
                    assert e.code == L.GS_ERR_BUDGET
        # argument validation: malformed calls return errors without touching a device
        assert lib.gs_project(None, None, 0, None, None, None) == L.GS_ERR_INVALID_ARG
        assert lib.gs_lod_select(None, None, 0, None, None) == L.GS_ERR_INVALID_ARG
        assert lib.gs_grads_zero(None, 0, None) == L.GS_ERR_INVALID_ARG
        go = L.GsGaussiansGrad()
        assert lib.gs_grads_zero(C.byref(go), 10, None) == L.GS_ERR_INVALID_ARG
        assert lib.gs_last_error()
        assert lib.gs_render_bwd_workspace_size(1000) > 0 and lib.gs_seg_workspace_size(100, 10000) > 0
        # server creation fails cleanly (no GPU here, or a bad configuration)
        scene = S.random_scene(64, seed=1)
        means = np.ascontiguousarray(scene.param_arrays()[0])
        g = L.GsGaussians()
        g.n = 64
        cfg = gs.ServeConfig(max_views_per_batch=2, n_streams=1, slot_capacity=1000, pair_capacity=1000,
                             pixel_capacity=4096, queue_capacity=4)
        srv = C.c_void_p()
        rc = lib.gs_serve_create(C.byref(g), C.byref(table.c()), C.byref(gs.RenderOptions().c()), C.byref(cfg.c()),
                                 0, C.byref(srv))
        assert rc != L.GS_OK
        for p in ("means", "scales", "quats", "opacities", "sh"):
            setattr(g, p, means.ctypes.data)
        bad = gs.ServeConfig(max_views_per_batch=99)
        assert lib.gs_serve_create(C.byref(g), C.byref(table.c()), C.byref(gs.RenderOptions().c()),
                                   C.byref(bad.c()), 0, C.byref(srv)) == L.GS_ERR_INVALID_ARG
        rc = lib.gs_serve_create(C.byref(g), C.byref(table.c()), C.byref(gs.RenderOptions().c()), C.byref(cfg.c()),
                                 0, C.byref(srv))
        if rc == L.GS_OK:
            assert lib.gs_serve_destroy(srv) == L.GS_OK
        print("ok", n_sel)
    """, rt)
    assert out.startswith("ok"), out
