"""Shared helpers of the GPU parity tests (HIP path vs FP64 oracle)."""
import numpy as np
import torch

from oracle import oracle as O
from synth import scenes

# FP32 vs FP64 forward tolerance: 1e-5 absolute on colour and alpha; depth is
# z-weighted (z up to ~10 m in these scenes), so its bound is 1e-5 relative to
# the largest visible depth.
TOL_C = 1e-5
TOL_A = 1e-5
TOL_D_REL = 1e-5
# gradients: relative L2 error per tensor
TOL_G = 1e-3


def dev_scene(s, device="cuda"):
    import paper_2405_19614_amd as gs
    g = gs.Gaussians.from_scene(s, device)
    poses = torch.tensor(np.asarray(s.poses, np.float32), device=device).reshape(s.V, 16).contiguous()
    return g, poses


def oracle_views(s, poses=None, bands=O.SMALL_BANDS):
    og = O.Gaussians.from_scene(s)
    poses = s.poses if poses is None else poses
    return og, O.render_views(og, s.cams, poses, bands=bands)


def forward_errors(s, color, depth, alpha, ref):
    """Max errors over the pixels the oracle does not flag as value-ambiguous
    (skip, termination or blend-order decisions within FP32 reach)."""
    ok = (ref["ambiguous"] & O.AMB_VALUE) == 0
    c = color.detach().cpu().numpy().astype(np.float64)
    d = depth.detach().cpu().numpy().astype(np.float64)
    a = alpha.detach().cpu().numpy().astype(np.float64)
    okc = np.concatenate([np.tile(ok[o:o + cm.npix], 3) for cm, o in zip(s.cams, s.pix_offsets()[:-1])])
    ec = np.abs(c - ref["color"])[okc].max(initial=0.0)
    ed = np.abs(d - ref["depth"])[ok].max(initial=0.0)
    ea = np.abs(a - ref["alpha"])[ok].max(initial=0.0)
    return ec, ed, ea, int((~ok).sum())


def zmax(s):
    return float(np.abs(s.means).max()) * 3.0 + 10.0


def rel(a, r):
    a = np.asarray(a, np.float64).reshape(-1)
    r = np.asarray(r, np.float64).reshape(-1)
    n = np.linalg.norm(r)
    return float(np.linalg.norm(a - r) / n) if n > 0 else float(np.linalg.norm(a))


def cotangents(s, ref, seed, scale=1.0):
    """Random upstream gradients, zero at pixels the oracle flags ambiguous
    (including the 0.99 clamp, which changes gradients)."""
    dC, dD, dA = scenes.random_cotangents(s, seed, scale)
    ok = (ref["ambiguous"] == 0).astype(np.float32)
    okc = np.concatenate([np.tile(ok[o:o + cm.npix], 3) for cm, o in zip(s.cams, s.pix_offsets()[:-1])])
    return dC * okc, dD * ok, dA * ok


GRAD_NAMES = ["means", "log_scales", "quats", "opacity_logits", "colors"]
