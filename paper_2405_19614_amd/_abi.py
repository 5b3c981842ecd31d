"""ctypes declarations of the C ABI in include/gs.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgs.so")

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_float = ctypes.c_float
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p
P_float = ctypes.POINTER(ctypes.c_float)

GS_OK, GS_EINVAL, GS_ENOMEM, GS_ECAPACITY, GS_EDEVICE, GS_ECAPTURE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "GS_OK", -1: "GS_EINVAL", -2: "GS_ENOMEM", -3: "GS_ECAPACITY", -4: "GS_EDEVICE",
                -5: "GS_ECAPTURE"}
MAX_VIEWS = 64
ABI_VERSION = 4     # GS_ABI_VERSION of include/gs.h


class gs_gaussians(ctypes.Structure):
    _fields_ = [("n", c_int64), ("sh_degree", c_int32), ("isotropic", c_int32), ("means", c_void_p),
                ("log_scales", c_void_p), ("quats", c_void_p), ("opacity_logits", c_void_p), ("colors", c_void_p)]


class gs_gaussian_grads(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p), ("opacity_logits", c_void_p),
                ("colors", c_void_p)]


class gs_camera(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("fx", c_float), ("fy", c_float), ("cx", c_float),
                ("cy", c_float)]


class gs_plan(ctypes.Structure):
    _fields_ = [("tile_w", c_int32), ("tile_h", c_int32), ("bin_w", c_int32), ("bin_h", c_int32),
                ("pair_capacity", c_int64), ("n_pairs", c_int64), ("n_visible", c_int64),
                ("bwd_tile_w", c_int32), ("bwd_tile_h", c_int32)]


class gs_step_opts(ctypes.Structure):
    _fields_ = [("w_color", c_float), ("w_depth", c_float), ("w_reproj", c_float), ("huber_delta", c_float),
                ("use_gate", c_int32), ("gate_gamma", c_float), ("update_gaussians", c_int32),
                ("update_poses", c_int32), ("accumulate_grads", c_int32), ("use_graph", c_int32),
                ("lr_means", c_float), ("lr_log_scales", c_float), ("lr_quats", c_float), ("lr_opacity", c_float),
                ("lr_colors", c_float), ("lr_pose", c_float), ("adam_b1", c_float), ("adam_b2", c_float),
                ("adam_eps", c_float), ("tile_w", c_int32), ("tile_h", c_int32), ("bin_w", c_int32),
                ("bin_h", c_int32), ("pair_capacity", c_int64), ("w_ssim", c_float),
                ("bwd_tile_w", c_int32), ("bwd_tile_h", c_int32)]


class gs_targets(ctypes.Structure):
    _fields_ = [("color", c_void_p), ("depth", c_void_p), ("mask", c_void_p)]


class gs_matches(ctypes.Structure):
    _fields_ = [("points", c_void_p), ("uv", c_void_p), ("view_idx", c_void_p), ("M", c_int64)]


class gs_adam(ctypes.Structure):
    _fields_ = [("m", c_void_p), ("v", c_void_p), ("step", c_void_p)]


EXPORTS = ["gs_abi_version", "gs_create", "gs_destroy", "gs_last_error", "gs_state_bytes", "gs_render_forward",
           "gs_render_forward_async",
           "gs_render_backward", "gs_reproj_residual", "gs_reproj_residual_noalloc", "gs_step_workspace_bytes", "gs_mapping_step",
           "gs_step_status", "gs_bin_records", "gs_autotune", "gs_set_tile", "gs_num_stages", "gs_stage_name",
           "gs_step_profile", "gs_set_pixels_per_thread", "gs_get_pixels_per_thread", "gs_set_bwd_shape", "gs_set_bin",
           "gs_ssim_workspace_bytes", "gs_ssim", "gs_prune_workspace_bytes", "gs_prune",
           "gs_densify_workspace_bytes", "gs_densify", "gs_select_viewpoints", "gs_adam_update", "gs_pose_retract",
           "gs_pose_tangent_grad"]

_lib = None


def load() -> ctypes.CDLL:
    """Load libgs.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2405_19614_amd/build.py "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    _lib = declare(ctypes.CDLL(LIB_PATH), LIB_PATH)
    return _lib


def declare(L: ctypes.CDLL, path: str) -> ctypes.CDLL:
    """Argument and result types of every export of a loaded build of the
    library (also used for instrumented builds in tests)."""
    PC = ctypes.POINTER(gs_camera)
    L.gs_abi_version.restype = c_int32
    if L.gs_abi_version() != ABI_VERSION:
        raise ImportError(f"{path} has ABI version {L.gs_abi_version()}, this binding needs {ABI_VERSION}: "
                          "rebuild it")
    L.gs_create.argtypes = [ctypes.POINTER(c_void_p), c_int32]
    L.gs_destroy.argtypes = [c_void_p]
    L.gs_destroy.restype = None
    L.gs_last_error.argtypes = [c_void_p]
    L.gs_last_error.restype = ctypes.c_char_p
    L.gs_state_bytes.argtypes = [PC, c_int32, c_int64, c_int64, c_int32, c_int32]
    L.gs_state_bytes.restype = c_size_t
    L.gs_step_workspace_bytes.argtypes = [PC, c_int32, c_int64, c_int32, c_int64, c_int32, c_int32]
    L.gs_step_workspace_bytes.restype = c_size_t
    L.gs_render_forward.argtypes = [c_void_p, ctypes.POINTER(gs_gaussians), PC, c_void_p, c_int32, c_void_p,
                                    c_void_p, c_void_p, c_void_p, c_size_t, ctypes.POINTER(gs_plan), c_void_p]
    L.gs_render_forward_async.argtypes = L.gs_render_forward.argtypes
    L.gs_render_backward.argtypes = [c_void_p, ctypes.POINTER(gs_gaussians), PC, c_void_p, c_int32, c_void_p,
                                     c_size_t, ctypes.POINTER(gs_plan), c_void_p, c_void_p, c_void_p,
                                     ctypes.POINTER(gs_gaussian_grads), c_void_p, c_void_p]
    L.gs_reproj_residual.argtypes = [c_void_p, PC, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_int64,
                                     c_float, c_float, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.gs_reproj_residual_noalloc.argtypes = L.gs_reproj_residual.argtypes
    L.gs_mapping_step.argtypes = [c_void_p, ctypes.POINTER(gs_gaussians), ctypes.POINTER(gs_gaussian_grads),
                                  ctypes.POINTER(gs_adam), PC, c_void_p, c_int32, ctypes.POINTER(gs_targets),
                                  ctypes.POINTER(gs_matches), ctypes.POINTER(gs_step_opts), c_void_p, c_size_t,
                                  c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.gs_step_status.argtypes = [c_void_p, c_void_p, c_size_t, ctypes.POINTER(c_int32), ctypes.POINTER(c_int64),
                                 ctypes.POINTER(c_int64), c_void_p]
    L.gs_bin_records.argtypes = [c_void_p, PC, c_int32, c_int64, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                 c_int64, c_void_p, ctypes.POINTER(c_int64), c_void_p, c_size_t, c_void_p]
    L.gs_autotune.argtypes = [c_void_p, ctypes.POINTER(gs_gaussians), PC, c_void_p, c_int32, c_int32,
                              ctypes.POINTER(c_int32), ctypes.POINTER(c_int32), ctypes.POINTER(c_int32),
                              ctypes.POINTER(c_int32), ctypes.POINTER(c_int32), ctypes.POINTER(c_int32), c_void_p]
    L.gs_set_bin.argtypes = [c_void_p, c_int32, c_int32]
    L.gs_set_tile.argtypes = [c_void_p, c_int32, c_int32]
    L.gs_set_pixels_per_thread.argtypes = [c_void_p, c_int32, c_int32, c_int32]
    L.gs_get_pixels_per_thread.argtypes = [c_void_p, c_int32, c_int32, c_int32]
    L.gs_set_bwd_shape.argtypes = [c_void_p, c_int32, c_int32, c_int32]
    PG = ctypes.POINTER(gs_gaussians)
    PA = ctypes.POINTER(gs_adam)
    L.gs_select_viewpoints.argtypes = [c_void_p, c_void_p, c_int32, ctypes.c_float, c_int32, c_void_p]
    L.gs_prune_workspace_bytes.argtypes = [c_int64]
    L.gs_prune_workspace_bytes.restype = c_size_t
    L.gs_prune.argtypes = [c_void_p, PG, ctypes.c_double, PG, PA, PA, c_int32, c_void_p, c_void_p, c_size_t, c_void_p]
    L.gs_densify_workspace_bytes.argtypes = [PC, c_int32]
    L.gs_densify_workspace_bytes.restype = c_size_t
    L.gs_densify.argtypes = [c_void_p, PC, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, ctypes.c_double, c_int32,
                             PG, c_int64, PA, PA, c_void_p, c_void_p, c_size_t, c_void_p]
    L.gs_ssim_workspace_bytes.argtypes = [PC, c_int32]
    L.gs_ssim_workspace_bytes.restype = c_size_t
    L.gs_ssim.argtypes = [c_void_p, PC, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                          c_size_t, c_void_p]
    L.gs_get_pixels_per_thread.restype = c_int32
    L.gs_num_stages.restype = c_int32
    L.gs_stage_name.argtypes = [c_int32]
    L.gs_stage_name.restype = ctypes.c_char_p
    L.gs_step_profile.argtypes = L.gs_mapping_step.argtypes[:-1] + [c_void_p, c_void_p, c_void_p]
    L.gs_adam_update.argtypes = [c_void_p, PG, ctypes.POINTER(gs_gaussian_grads), PA, c_void_p, c_void_p, c_int32,
                                 ctypes.POINTER(gs_step_opts), c_void_p]
    L.gs_pose_retract.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]
    L.gs_pose_tangent_grad.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]
    return L
