"""Sanitizer builds of the CPU-side code (AddressSanitizer + UndefinedBehaviorSanitizer).

* The oracle (``oracle/gs_oracle.c``) built by gcc with -fsanitize=address,undefined
  runs projection, whole-image and pixel-list rendering, the reverse mode,
  binning, the re-projection residual and the SH basis over scenes that reach
  every branch (clamped alpha, the 1e-4 stop, the Jacobian clamp, the near
  plane, SH colour) and the degenerate sizes (no Gaussian, a 1x1 image); its
  results equal the normal build's.
* The library's host code (``csrc/abi.cpp``, sanitizers on the host pass only,
  through -Xarch_host), linked with the normal kernel objects, runs every
  entry point's host-side path that needs no device: sizing, argument
  validation, the viewpoint rule, context creation without a device.

Each runs in a child process with its sanitizer runtime preloaded; any report
ends that process with a non-zero status.
"""
import glob
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(script, env_extra, preload, tmp_path):
    env = dict(os.environ)
    env.update(SAN_ENV)
    env.update(env_extra)
    env["LD_PRELOAD"] = preload
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    env["OMP_NUM_THREADS"] = "2"
    p = subprocess.run([sys.executable, "-c", textwrap.dedent(script)], env=env, cwd=str(tmp_path),
                       capture_output=True, text=True, timeout=600)
    assert p.returncode == 0, f"exit {p.returncode}\n{p.stdout[-4000:]}\n{p.stderr[-6000:]}"
    return p.stdout


ORACLE_SCRIPT = """
    import sys, numpy as np
    from oracle import oracle as O
    from synth import scenes
    out = {}
    rng = np.random.default_rng(3)

    def scene(n, W, H, sh, front=0.0):
        means = np.stack([rng.uniform(-0.9, 0.9, n), rng.uniform(-0.7, 0.7, n), rng.uniform(-0.5, 4.0, n)], 1)
        means[: n // 8, 0] *= 4.0                       # far off-axis: the Jacobian clamp
        means[n // 8: n // 4, 2] = rng.uniform(0.1, 0.3, n // 8)   # about the near plane
        ls = rng.normal(-2.4, 0.6, (n, 3))
        q = rng.standard_normal((n, 4))
        opl = rng.normal(1.0, 2.5, n)
        opl[: n // 6] = rng.uniform(5.0, 9.0, n // 6)   # alpha clamped at 0.99, early stops
        K = 1 if sh < 0 else (sh + 1) ** 2
        col = rng.uniform(0, 1, (n, 3)) if sh < 0 else rng.normal(0, 0.3, (n, K, 3))
        cam = scenes.Camera(W, H, 0.9 * W, 0.9 * W, W / 2 - 0.3, H / 2 + 0.2)
        T = O.se3_exp(rng.normal(0, 0.05, 6))
        return O.Gaussians(means, ls, q, opl, col, sh), cam, T

    cases = {"rgb": scene(120, 40, 30, -1), "sh3": scene(90, 33, 21, 3), "one_pixel": scene(40, 1, 1, -1),
             "empty": scene(0, 16, 12, -1)}
    for name, (g, cam, T) in cases.items():
        out[name + "_proj"] = O.project(g, cam, T)
        r = O.render(g, cam, T)
        for k in ("color", "depth", "alpha", "tfinal", "order_bound"):
            out[f"{name}_{k}"] = r[k]
        out[name + "_amb"] = r["ambiguous"].astype(np.int64)
        px = np.stack([rng.integers(0, cam.width, 7), rng.integers(0, cam.height, 7)], 1)
        out[name + "_pix"] = O.render(g, cam, T, pixels=px)["color"]
        dC = rng.standard_normal(3 * cam.width * cam.height)
        dD = rng.standard_normal(cam.width * cam.height)
        dA = rng.standard_normal(cam.width * cam.height)
        gr = O.backward(g, cam, T, dC, dD, dA)
        for k, v in gr.items():
            out[f"{name}_grad_{k}"] = np.asarray(v)
    # binning of synthetic records with ties and empty rects
    sizes = [(40, 30), (1, 1), (17, 9)]
    n = 50
    rect = np.zeros((len(sizes) * n, 2), np.uint32)
    depth = rng.choice([1.0, 1.5, 2.0, 3.25], len(sizes) * n)
    for v, (w, h) in enumerate(sizes):
        x0 = rng.integers(0, w, n); x1 = np.minimum(x0 + rng.integers(-1, 12, n), w - 1)
        y0 = rng.integers(0, h, n); y1 = np.minimum(y0 + rng.integers(-1, 12, n), h - 1)
        rect[v * n:(v + 1) * n, 0] = x0 | (x1 << 16)
        rect[v * n:(v + 1) * n, 1] = y0 | (y1 << 16)
    vals, ranges = O.binning(sizes, n, 8, 8, rect, depth)
    out["bin_vals"] = np.asarray(vals, np.int64)
    out["bin_ranges"] = np.asarray(ranges, np.int64)
    # re-projection with matches behind the near plane
    s = scenes.c4(n=2000, views=3, res_scale=0.3, vis_range=(200, 2000), matches=(20, 40), seed=9)
    rp = O.reproj(s.cams, s.poses, s.points, s.uv, s.view_idx, 2.0)
    for k, v in rp.items():
        out["reproj_" + k] = np.asarray(v)
    dirs = rng.standard_normal((50, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    out["sh"] = np.asarray(O.sh_basis(3, dirs))
    np.savez(sys.argv[1] if len(sys.argv) > 1 else "oracle_out.npz", **out)
    print("ORACLE_DONE")
"""


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
                           "-ffp-contract=off", "-fno-fast-math", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           os.path.join(ROOT, "oracle", "gs_oracle.c"), "-o", lib, "-lm"])
    # the same script with the instrumented build (child) and the normal one (here)
    stdout = _run(ORACLE_SCRIPT, {"GS_ORACLE_LIB": lib}, asan, tmp_path)
    assert "ORACLE_DONE" in stdout
    san = np.load(tmp_path / "oracle_out.npz")
    ref_dir = tmp_path / "ref"
    ref_dir.mkdir()
    env = dict(os.environ, PYTHONPATH=ROOT, OMP_NUM_THREADS="2")
    env.pop("GS_ORACLE_LIB", None)
    subprocess.check_call([sys.executable, "-c", textwrap.dedent(ORACLE_SCRIPT), str(ref_dir / "o.npz")], env=env,
                          cwd=str(ref_dir))
    ref = np.load(ref_dir / "o.npz")
    assert sorted(san.files) == sorted(ref.files)
    for k in ref.files:
        np.testing.assert_allclose(san[k], ref[k], rtol=1e-12, atol=1e-12, err_msg=k)


HOST_SCRIPT = """
    import ctypes, sys
    import numpy as np
    from paper_2405_19614_amd import _abi as A
    L = A.declare(ctypes.CDLL(sys.argv[1]), sys.argv[1])
    cams = (A.gs_camera * 3)(A.gs_camera(64, 48, 60, 60, 32, 24), A.gs_camera(70, 45, 60, 60, 35, 22.5),
                             A.gs_camera(1, 1, 2, 2, 0, 0))
    for V in (1, 2, 3):
        for n in (0, 1, 63, 64, 65, 1000):
            for cap in (0, 1, 5000):
                for bw, bh in ((0, 0), (8, 8), (64, 64), (512, 256), (12, 12), (4096, 8)):
                    L.gs_state_bytes(cams, V, n, cap, bw, bh)
                    L.gs_step_workspace_bytes(cams, V, n, 3, cap, bw, bh)
    for bad in (0, -1, 65):
        assert L.gs_state_bytes(cams, bad, 10, 10, 16, 16) == 0
    assert L.gs_state_bytes(None, 1, 10, 10, 16, 16) == 0
    assert L.gs_ssim_workspace_bytes(cams, 3) > 0 and L.gs_ssim_workspace_bytes(cams, 0) == 0
    assert L.gs_densify_workspace_bytes(cams, 3) > 0
    assert L.gs_prune_workspace_bytes(0) > 0 and L.gs_prune_workspace_bytes(-5) == 0
    # the viewpoint rule on random covisibility, and its argument checks
    rng = np.random.default_rng(7)
    for trial in range(40):
        F = int(rng.integers(1, 30))
        covis = np.ascontiguousarray(rng.integers(0, 150, (F, F)).astype(np.int32))
        nobs = np.ascontiguousarray(rng.integers(0, 200, F).astype(np.int32))
        sel = np.zeros(F, np.int32)
        rc = L.gs_select_viewpoints(covis.ctypes.data_as(ctypes.c_void_p), nobs.ctypes.data_as(ctypes.c_void_p), F,
                                    0.75, 20, sel.ctypes.data_as(ctypes.c_void_p))
        assert rc >= 0
    assert L.gs_select_viewpoints(None, None, -1, 0.75, 20, None) == A.GS_EINVAL
    # every entry point rejects a missing context before touching a device
    plan = A.gs_plan(16, 16, 64, 64, 0, 0, 0)
    assert L.gs_render_forward(None, None, None, None, 1, None, None, None, None, 0, ctypes.byref(plan), None) \
        == A.GS_EINVAL
    assert L.gs_render_forward_async(None, None, None, None, 1, None, None, None, None, 0, ctypes.byref(plan),
                                     None) == A.GS_EINVAL
    assert L.gs_set_tile(None, 16, 16) == A.GS_EINVAL
    assert L.gs_set_bwd_shape(None, 32, 32, 4) == A.GS_EINVAL
    assert L.gs_get_pixels_per_thread(None, 0, 16, 16) == A.GS_EINVAL
    assert L.gs_ssim(None, cams, 2, None, None, None, None, None, None, 0, None) == A.GS_EINVAL
    for k in range(L.gs_num_stages()):
        assert L.gs_stage_name(k)
    # a context needs a device: without one, creation fails with a message
    h = ctypes.c_void_p()
    rc = L.gs_create(ctypes.byref(h), 0)
    msg = L.gs_last_error(None)
    print("create:", rc, msg)
    if rc == 0:
        L.gs_destroy(h)
    print("HOST_DONE")
"""


def _clang_asan():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    rt = _clang_asan()
    if rt is None or not os.path.exists(HIPCC):
        pytest.skip("no hipcc AddressSanitizer runtime")
    build_dir = os.path.join(ROOT, "_build")
    kernels = ["project", "binning", "raster", "step", "ssim", "maintain"]
    if not all(os.path.exists(os.path.join(build_dir, k + ".o")) for k in kernels):
        from paper_2405_19614_amd import build
        build.build()
    inc = [f"-I{os.path.join(ROOT, 'include')}", f"-I{os.path.join(ROOT, 'paper_2405_19614_amd', 'csrc')}"]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    obj = str(tmp_path / "abi_san.o")
    lib = str(tmp_path / "libgs_san.so")
    # the host pass of abi.cpp instrumented; its device pass (the static
    # scratch array) and the kernel objects as in the normal build
    subprocess.check_call([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-x", "hip", *san,
                           *inc, "-c", os.path.join(ROOT, "paper_2405_19614_amd", "csrc", "abi.cpp"), "-o", obj],
                          stderr=subprocess.DEVNULL)
    subprocess.check_call([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *san, obj,
                           *[os.path.join(build_dir, k + ".o") for k in kernels], "-o", lib],
                          stderr=subprocess.DEVNULL)
    stdout = _run(HOST_SCRIPT.replace("sys.argv[1]", repr(lib)), {}, rt, tmp_path)
    print(stdout)
    assert "HOST_DONE" in stdout
