"""Host-side checks of the C-ABI library (no GPU needed, no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gs.h")
LIB = os.path.join(ROOT, "paper_2405_19614_amd", "libgs.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2405_19614_amd import build
        build.build()
    from paper_2405_19614_amd import _abi
    return _abi.load()


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ["gs_render_forward", "gs_render_backward", "gs_reproj_residual", "gs_mapping_step",
                     "gs_create", "gs_destroy", "gs_last_error", "gs_abi_version"]:
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_python_binding_names_every_export(lib):
    from paper_2405_19614_amd import _abi
    assert sorted(_abi.EXPORTS) == _declared()


def test_abi_version(lib):
    assert lib.gs_abi_version() == 4


def test_null_context_rejected_without_device_work(lib):
    from paper_2405_19614_amd import _abi as A
    plan = A.gs_plan(16, 16, 64, 64, 0, 0, 0)
    rc = lib.gs_render_forward(None, None, None, None, 1, None, None, None, None, 0, ctypes.byref(plan), None)
    assert rc == A.GS_EINVAL
    assert lib.gs_set_tile(None, 16, 16) == A.GS_EINVAL
    assert lib.gs_get_pixels_per_thread(None, 0, 16, 16) == A.GS_EINVAL
    assert lib.gs_set_bwd_shape(None, 32, 32, 4) == A.GS_EINVAL


def test_state_bytes_validation(lib):
    from paper_2405_19614_amd import _abi as A
    cams = (A.gs_camera * 2)(A.gs_camera(64, 48, 60, 60, 32, 24), A.gs_camera(70, 45, 60, 60, 35, 22.5))
    ok = lib.gs_state_bytes(cams, 2, 1000, 10000, 16, 16)
    assert ok > 0
    # monotone in every size
    assert lib.gs_state_bytes(cams, 2, 2000, 10000, 16, 16) > ok
    assert lib.gs_state_bytes(cams, 2, 1000, 20000, 16, 16) > ok
    # invalid: bin not a multiple of 8, V = 0, V too large, negative n, bad camera, capacity too large
    assert lib.gs_state_bytes(cams, 2, 1000, 10000, 12, 12) == 0
    assert lib.gs_state_bytes(cams, 0, 1000, 10000, 16, 16) == 0
    assert lib.gs_state_bytes(cams, 65, 1000, 10000, 16, 16) == 0
    assert lib.gs_state_bytes(cams, 2, -1, 10000, 16, 16) == 0
    assert lib.gs_state_bytes(cams, 2, 1000, 1 << 31, 16, 16) == 0
    bad = (A.gs_camera * 1)(A.gs_camera(0, 48, 60, 60, 32, 24))
    assert lib.gs_state_bytes(bad, 1, 10, 10, 16, 16) == 0
    bad = (A.gs_camera * 1)(A.gs_camera(64, 48, -1.0, 60, 32, 24))
    assert lib.gs_state_bytes(bad, 1, 10, 10, 16, 16) == 0
    assert lib.gs_state_bytes(None, 1, 10, 10, 16, 16) == 0
    # the workspace holds the state plus the loss buffers
    assert lib.gs_step_workspace_bytes(cams, 2, 1000, -1, 10000, 16, 16) > ok


def test_bin_shapes_accepted(lib):
    from paper_2405_19614_amd import _abi as A
    cams = (A.gs_camera * 1)(A.gs_camera(64, 48, 60, 60, 32, 24))
    for bw, bh in [(16, 16), (16, 8), (8, 8), (32, 8), (32, 16), (64, 64), (128, 64), (2048, 2048), (0, 0)]:
        assert lib.gs_state_bytes(cams, 1, 10, 10, bw, bh) > 0
    for bw, bh in [(4, 8), (8, 12), (4096, 8)]:
        assert lib.gs_state_bytes(cams, 1, 10, 10, bw, bh) == 0


def test_ssim_workspace_sizing(lib):
    from paper_2405_19614_amd import _abi as A
    cams = (A.gs_camera * 2)(A.gs_camera(64, 48, 60, 60, 32, 24), A.gs_camera(33, 17, 60, 60, 16, 8))
    npx = 64 * 48 + 33 * 17
    tiles = 2 * 3 + 2 * 2   # 32 x 16 SSIM tiles per view
    b = lib.gs_ssim_workspace_bytes(cams, 2)
    assert b >= 9 * 4 * npx + 3 * 8 * tiles
    assert lib.gs_ssim_workspace_bytes(cams, 0) == 0
    assert lib.gs_ssim(None, cams, 2, None, None, None, None, None, None, 0, None) == A.GS_EINVAL


def test_paper_mapping_preset_matches_table():
    """The mapping preset is the paper's (1 - zeta)(w4 L1_D + w5 L1_C) + zeta L_SSIM."""
    import json
    from paper_2405_19614_amd.binding import PAPER_MAPPING
    hp = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_hyperparams.json")))["values"]
    z = hp["zeta"]
    assert abs(PAPER_MAPPING["w_ssim"] - z) < 1e-12
    assert abs(PAPER_MAPPING["w_color"] - (1 - z) * hp["w5"]) < 1e-12
    assert abs(PAPER_MAPPING["w_depth"] - (1 - z) * hp["w4"]) < 1e-12


def test_paper_preset_matches_table():
    """The Fusion Bridge preset of the binding equals the paper's table."""
    import json
    from paper_2405_19614_amd.binding import PAPER_FUSION_BRIDGE
    hp = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_hyperparams.json")))["values"]
    assert PAPER_FUSION_BRIDGE["w_reproj"] == hp["w1"]
    assert PAPER_FUSION_BRIDGE["w_color"] == hp["w2"]
    assert PAPER_FUSION_BRIDGE["w_depth"] == hp["w3"]
    assert PAPER_FUSION_BRIDGE["gate_gamma"] == hp["gamma"]


def test_viewpoint_selection_matches_oracle(lib):
    """The library's host rule equals the oracle's on random covisibility."""
    import numpy as np
    from oracle import oracle as O
    from paper_2405_19614_amd import select_viewpoints
    rng = np.random.default_rng(21)
    for trial in range(50):
        F = int(rng.integers(1, 40))
        covis = rng.integers(0, 150, (F, F)).astype(np.int32)
        n_obs = rng.integers(0, 200, F).astype(np.int32)
        alpha, beta = float(rng.choice([0.5, 0.75, 0.9])), int(rng.choice([5, 20, 40]))
        got = select_viewpoints(covis, n_obs, alpha, beta)
        want = O.select_viewpoints(covis, n_obs, alpha, beta)
        assert list(got) == list(want), trial
    # boundaries: M == beta selected, M == alpha * T not
    covis = np.array([[0, 20, 0], [0, 0, 0], [0, 0, 0]], np.int32)
    covis[1, 2] = 75
    assert list(select_viewpoints(covis, np.array([100, 100, 0], np.int32), 0.75, 20)) == [True, True, False]
    from paper_2405_19614_amd import _abi as A
    assert lib.gs_select_viewpoints(None, None, -1, 0.75, 20, None) == A.GS_EINVAL
    assert lib.gs_select_viewpoints(None, None, 0, 0.75, 20, None) == 0
