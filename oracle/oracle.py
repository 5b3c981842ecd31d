"""FP64 oracle for the Gaussian-splatting hot path (Python side).

TEST INFRASTRUCTURE ONLY: only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module.  It shares no code
with the HIP path and never imports it.

The per-view renderer, its reverse mode, the re-projection residual and the
binning definition live in ``gs_oracle.c`` (plain C, FP64, OpenMP).  This
module marshals numpy arrays into it and adds the parts that are a few lines
of numpy:

* the loss of the joint optimisation (Sec. 3.3, joint-loss equation) and the
  L1 terms of the mapping loss (Sec. 3.4, mapping-loss equation), as means per
  view averaged over views, with an optional constant pixel mask and the
  filter gate of Sec. 3.3 (gate equation);
* the paper's own eight-parameter isotropic Gaussian (Sec. 3.4 "Gaussian
  Representation") as the anisotropic one with equal scales, and the reverse
  mode of that map;
* the SSIM term of the mapping loss (Sec. 3.4, mapping-loss equation) on the
  RGB render, with its gradient;
* Gaussian pruning and densification (Sec. 3.4), with the re-layout of the
  Adam moments they imply;
* SE(3) exponential for the left-perturbation pose tangent xi = (v, w);
* Adam (the paper says only "gradient-based optimization", Sec. 3.4).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GS_ORACLE_LIB names another build of gs_oracle.c to load instead (the
# sanitizer test's instrumented one); it is then used as it is
_LIB_PATH = os.environ.get("GS_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "gs_oracle.c")

# decision bands for flagging pixels whose result an FP32 renderer may
# legitimately decide the other way: relative for the 1/255 skip and the 1e-4
# termination, absolute for the 0.99 clamp, and for the blend order of two
# Gaussians a multiple of the single-precision unit roundoff (2^-24) times
# the magnitude of the terms of the depth dot product.  The defaults cover
# images up to ~1200 px wide, where FP32 projected means carry ~1e-4 px of
# rounding; SMALL_BANDS suit images of a few hundred pixels.
BAND_SKIP = 2e-4
BAND_CLAMP = 2e-4
BAND_TERM = 5e-4
BAND_ORDER = 8 * 2.0 ** -24
BANDS = (BAND_SKIP, BAND_CLAMP, BAND_TERM, BAND_ORDER)
SMALL_BANDS = (5e-5, 5e-5, 2e-4, BAND_ORDER)
# flag bits: the 1/255 skip, the 0.99 clamp, the 1e-4 stop near their
# thresholds; a blend order within FP32 depth rounding (a tie); a tie at the
# candidate that stops the pixel
AMB_SKIP, AMB_CLAMP, AMB_TERM, AMB_ORDER, AMB_ORDER_STOP = 1, 2, 4, 8, 16
AMB_VALUE = AMB_SKIP | AMB_TERM | AMB_ORDER | AMB_ORDER_STOP   # decisions that change rendered values
# decisions whose effect the oracle does not bound; a pixel flagged only
# AMB_ORDER and / or AMB_ORDER_STOP is bounded by render()["order_bound"]
AMB_UNBOUNDED = AMB_SKIP | AMB_TERM


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP, no FP contraction)."""
    if os.environ.get("GS_ORACLE_LIB"):
        return _LIB_PATH
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        L.or_project.argtypes = [i64, ctypes.c_int] + [ctypes.c_void_p] * 5 + [ctypes.c_int, ctypes.c_int] + \
            [ctypes.c_double] * 4 + [ctypes.c_void_p, ctypes.c_void_p]
        L.or_render.argtypes = [i64, ctypes.c_int] + [ctypes.c_void_p] * 5 + [ctypes.c_int, ctypes.c_int] + \
            [ctypes.c_double] * 4 + [ctypes.c_void_p, i64, ctypes.c_void_p] + [ctypes.c_double] * 4 + \
            [ctypes.c_void_p] * 8
        L.or_backward.argtypes = [i64, ctypes.c_int] + [ctypes.c_void_p] * 5 + [ctypes.c_int, ctypes.c_int] + \
            [ctypes.c_double] * 4 + [ctypes.c_void_p, i64, ctypes.c_void_p] + [ctypes.c_void_p] * 3 + \
            [ctypes.c_void_p] * 6
        L.or_reproj.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 4 + [i64] + [ctypes.c_void_p] * 3 + \
            [ctypes.c_double] + [ctypes.c_void_p] * 4
        L.or_binning_count.argtypes = [ctypes.c_int, i64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_void_p]
        L.or_binning_count.restype = i64
        L.or_binning.argtypes = [ctypes.c_int, i64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, i64]
        L.or_sh_basis.argtypes = [ctypes.c_int, i64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.or_num_threads.restype = ctypes.c_int
        del dp
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on."""
    lib().or_set_num_threads(int(n))


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Gaussians:
    """FP64 copies of the Gaussian parameters (promoted from the FP32 inputs)."""

    def __init__(self, means, log_scales, quats, opacity_logits, colors, sh_degree: int = -1):
        self.means = _d(means).reshape(-1, 3)
        self.log_scales = _d(log_scales).reshape(-1, 3)
        self.quats = _d(quats).reshape(-1, 4)
        self.opacity_logits = _d(opacity_logits).reshape(-1)
        self.sh_degree = int(sh_degree)
        K = 1 if sh_degree < 0 else (sh_degree + 1) ** 2
        self.colors = _d(colors).reshape(-1, 3) if sh_degree < 0 else _d(colors).reshape(-1, K, 3)
        self.n = self.means.shape[0]

    @classmethod
    def from_scene(cls, s) -> "Gaussians":
        if getattr(s, "isotropic", False):
            return from_isotropic(s.means, s.log_scales, s.opacity_logits, s.colors, s.sh_degree)
        return cls(s.means, s.log_scales, s.quats, s.opacity_logits, s.colors, s.sh_degree)

    def args(self):
        return (self.n, self.sh_degree, _p(self.means), _p(self.log_scales), _p(self.quats),
                _p(self.opacity_logits), _p(self.colors))


def from_isotropic(means, log_radius, opacity_logits, colors, sh_degree: int = -1) -> Gaussians:
    """The paper's eight-parameter Gaussian (Sec. 3.4 "Gaussian
    Representation", Eq. gauss): centre mu, one radius r = exp(log_radius),
    opacity and colour, f(x) = o exp(-|x - mu|^2 / (2 r^2)).  Its covariance
    r^2 I is that of the anisotropic Gaussian with scale r on every axis,
    whatever the rotation: the returned parameters hold log r on each axis and
    the identity quaternion."""
    lr = _d(log_radius).reshape(-1)
    n = lr.shape[0]
    return Gaussians(means, np.repeat(lr[:, None], 3, axis=1), np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)),
                     opacity_logits, colors, sh_degree)


def isotropic_grads(grads: Dict[str, np.ndarray]) -> Dict[str, np.ndarray]:
    """Reverse mode of ``from_isotropic``: log r feeds all three log-scales,
    so its gradient is their sum; the quaternion is a constant there."""
    out = {k: v for k, v in grads.items() if k not in ("log_scales", "quats")}
    out["log_radius"] = np.asarray(grads["log_scales"]).sum(axis=1)
    return out


def _cam_args(cam, T):
    T = _d(T).reshape(4, 4)
    return (int(cam.width), int(cam.height), float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)), T


def project(g: Gaussians, cam, T) -> np.ndarray:
    """Per-Gaussian records [n,20]: valid, u, v, A, B, C, o, r, g, b, z,
    radius, x0, x1, y0, y1, a, b, c, det."""
    ca, T = _cam_args(cam, T)
    out = np.zeros((g.n, 20), np.float64)
    lib().or_project(*g.args(), *ca, _p(T), _p(out))
    return out


def render(g: Gaussians, cam, T, pixels: Optional[np.ndarray] = None, bands=BANDS) -> Dict[str, np.ndarray]:
    """Render one view (whole image, or the pixels [k,2] (x, y) listed).

    Returns color [3,H,W] (or [3,k]), depth, alpha, tfinal, nblend,
    ambiguous (int8 flags), order_bound [5,...] (the largest change of the
    three colour channels, the depth and the alpha that reordering near-tied
    blended Gaussians can make) and nfrag (candidates visited)."""
    ca, T = _cam_args(cam, T)
    if pixels is None:
        shape = (cam.height, cam.width)
        npix, pix = -1, None
        np_ = cam.width * cam.height
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
        npix = np_ = pix.shape[0]
        shape = (np_,)
    color = np.zeros(3 * np_, np.float64)
    depth = np.zeros(np_, np.float64)
    alpha = np.zeros(np_, np.float64)
    tfin = np.zeros(np_, np.float64)
    nbl = np.zeros(np_, np.int32)
    amb = np.zeros(np_, np.int8)
    nfrag = np.zeros(1, np.int64)
    bound = np.zeros(5 * np_, np.float64)
    b4 = tuple(bands) + ((BAND_ORDER,) if len(bands) == 3 else ())
    rc = lib().or_render(*g.args(), *ca, _p(T), npix, _p(pix), *(float(b) for b in b4), _p(color), _p(depth),
                         _p(alpha), _p(tfin), _p(nbl), _p(amb), _p(nfrag), _p(bound))
    if rc != 0:
        raise MemoryError("oracle render failed")
    return {"color": color.reshape((3,) + shape), "depth": depth.reshape(shape), "alpha": alpha.reshape(shape),
            "tfinal": tfin.reshape(shape), "nblend": nbl.reshape(shape), "ambiguous": amb.reshape(shape),
            "order_bound": bound.reshape((5,) + shape), "nfrag": int(nfrag[0])}


def backward(g: Gaussians, cam, T, dC=None, dD=None, dA=None, pixels: Optional[np.ndarray] = None,
             grads: Optional[Dict[str, np.ndarray]] = None) -> Dict[str, np.ndarray]:
    """Reverse mode of ``render`` for one view.  Accumulates into ``grads``
    (created if None): means, log_scales, quats, opacity_logits, colors, pose
    (the 6-vector d/dxi of T <- Exp(xi) T at xi = 0)."""
    ca, T = _cam_args(cam, T)
    if pixels is None:
        npix, pix = -1, None
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
        npix = pix.shape[0]
    if grads is None:
        grads = {"means": np.zeros_like(g.means), "log_scales": np.zeros_like(g.log_scales),
                 "quats": np.zeros_like(g.quats), "opacity_logits": np.zeros_like(g.opacity_logits),
                 "colors": np.zeros_like(g.colors), "pose": np.zeros(6)}
    dC = None if dC is None else _d(dC).reshape(-1)
    dD = None if dD is None else _d(dD).reshape(-1)
    dA = None if dA is None else _d(dA).reshape(-1)
    rc = lib().or_backward(*g.args(), *ca, _p(T), npix, _p(pix), _p(dC), _p(dD), _p(dA), _p(grads["means"]),
                           _p(grads["log_scales"]), _p(grads["quats"]), _p(grads["opacity_logits"]),
                           _p(grads["colors"]), _p(grads["pose"]))
    if rc != 0:
        raise MemoryError("oracle backward failed")
    return grads


def render_views(g: Gaussians, cams, poses, bands=BANDS) -> Dict[str, np.ndarray]:
    """All views, flattened in the library's ragged layout: color is the
    concatenation of each view's planar [3,H,W]; depth/alpha/tfinal of each
    view's [H,W]."""
    outs = [render(g, c, poses[v], bands=bands) for v, c in enumerate(cams)]
    return {"color": np.concatenate([o["color"].reshape(-1) for o in outs]),
            "depth": np.concatenate([o["depth"].reshape(-1) for o in outs]),
            "alpha": np.concatenate([o["alpha"].reshape(-1) for o in outs]),
            "tfinal": np.concatenate([o["tfinal"].reshape(-1) for o in outs]),
            "ambiguous": np.concatenate([o["ambiguous"].reshape(-1) for o in outs]),
            "nblend": np.concatenate([o["nblend"].reshape(-1) for o in outs]),
            "order_bound": np.concatenate([o["order_bound"].reshape(5, -1) for o in outs], axis=1),
            "nfrag": sum(o["nfrag"] for o in outs)}


def backward_views(g: Gaussians, cams, poses, dC, dD, dA) -> Dict[str, np.ndarray]:
    """Reverse mode of ``render_views`` with flat ragged cotangents; returns
    Gaussian gradients summed over views and pose [V,6]."""
    grads = None
    pose = np.zeros((len(cams), 6))
    co = cd = 0
    for v, c in enumerate(cams):
        P = c.width * c.height
        sl3 = None if dC is None else dC[co:co + 3 * P]
        sl = None if dD is None else dD[cd:cd + P]
        sa = None if dA is None else dA[cd:cd + P]
        if grads is not None:
            grads["pose"] = np.zeros(6)
        grads = backward(g, c, poses[v], sl3, sl, sa, grads=grads)
        pose[v] = grads["pose"]
        co += 3 * P
        cd += P
    grads["pose"] = pose
    return grads


def reproj(cams, poses, points, uv, view_idx, delta: float) -> Dict[str, np.ndarray]:
    """Sec. 3.2 Eq. lba residuals with a Huber kernel; per-view mean loss and
    its pose gradient."""
    V = len(cams)
    W = np.array([c.width for c in cams], np.int32)
    H = np.array([c.height for c in cams], np.int32)
    intr = _d([[c.fx, c.fy, c.cx, c.cy] for c in cams]).reshape(V, 4)
    T = _d(poses).reshape(V, 16)
    P = _d(points).reshape(-1, 3)
    U = _d(uv).reshape(-1, 2)
    vid = np.ascontiguousarray(view_idx, dtype=np.int32)
    M = P.shape[0]
    res = np.zeros((M, 2))
    loss = np.zeros(V)
    dpose = np.zeros((V, 6))
    nvalid = np.zeros(V, np.int64)
    lib().or_reproj(V, _p(W), _p(H), _p(intr), _p(T), M, _p(P), _p(U), _p(vid), float(delta), _p(res), _p(loss),
                    _p(dpose), _p(nvalid))
    return {"residual": res, "loss": loss, "dpose": dpose, "nvalid": nvalid}


def reproj_point_grads(cams, poses, points, uv, view_idx, delta: float, weight: float = 1.0) -> np.ndarray:
    """d/dP of weight * sum_v (mean over view v's valid matches of h(|r|)),
    the point side of the full bundle adjustment (Sec. 3.2 Eq. for:ba):
    p = R P + t, r = uv - pi(p), dh/dr = r (|r| <= delta) or delta r / |r|,
    dr/dp = -[[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]], dp/dP = R."""
    P = _d(points).reshape(-1, 3)
    U = _d(uv).reshape(-1, 2)
    vid = np.asarray(view_idx).reshape(-1)
    V = len(cams)
    out = np.zeros_like(P)
    valid = np.zeros(len(P), bool)
    for m in range(len(P)):
        v = int(vid[m])
        if v < 0 or v >= V:
            continue
        T = _d(poses[v]).reshape(4, 4)
        p = T[:3, :3] @ P[m] + T[:3, 3]
        if not p[2] > 0.2:
            continue
        c = cams[v]
        r = U[m] - np.array([c.fx * p[0] / p[2] + c.cx, c.fy * p[1] / p[2] + c.cy])
        e = np.linalg.norm(r)
        dh_dr = r if e <= delta else delta * r / e
        J = np.array([[c.fx / p[2], 0.0, -c.fx * p[0] / p[2] ** 2], [0.0, c.fy / p[2], -c.fy * p[1] / p[2] ** 2]])
        out[m] = -(dh_dr @ J) @ T[:3, :3]
        valid[m] = True
    for v in range(V):
        sel = valid & (vid == v)
        if sel.any():
            out[sel] *= weight / sel.sum()
    return out


def select_viewpoints(covis, n_obs, alpha: float, beta: int) -> np.ndarray:
    """Sec. 3.3 selection equation over keyframes in time order: the first
    is selected; keyframe i is selected when beta <= M < alpha T, M = feature
    matches between i and the previous selected keyframe p, T = matched map
    points observed by p."""
    F = len(n_obs)
    sel = np.zeros(F, bool)
    if F == 0:
        return sel
    sel[0] = True
    prev = 0
    for i in range(1, F):
        M = int(covis[prev][i])
        if beta <= M and M < alpha * float(n_obs[prev]):
            sel[i] = True
            prev = i
    return sel


def binning(sizes, n: int, tile_w: int, tile_h: int, rect: np.ndarray, depth: np.ndarray):
    """Definition of the (tile, depth, record) binning: returns (values,
    ranges) where values lists record ids sorted by (global tile, FP32 depth
    bits, record) and ranges [T,2] holds each tile's [start, end), (0, 0)
    when empty."""
    V = len(sizes)
    W = np.array([s[0] for s in sizes], np.int32)
    H = np.array([s[1] for s in sizes], np.int32)
    rect = np.ascontiguousarray(rect, dtype=np.uint32).reshape(-1, 2)
    depth = np.ascontiguousarray(depth, dtype=np.float32).reshape(-1)
    total = int(lib().or_binning_count(V, n, _p(W), _p(H), tile_w, tile_h, _p(rect)))
    ntiles = int(sum(((w + tile_w - 1) // tile_w) * ((h + tile_h - 1) // tile_h) for w, h in sizes))
    values = np.zeros(max(total, 1), np.uint32)
    ranges = np.zeros((ntiles, 2), np.uint32)
    lib().or_binning(V, n, _p(W), _p(H), tile_w, tile_h, _p(rect), _p(depth), _p(values), _p(ranges), ntiles)
    return values[:total], ranges


def sh_basis(deg: int, dirs: np.ndarray, grad: bool = False):
    dirs = _d(dirs).reshape(-1, 3)
    K = (deg + 1) ** 2
    Y = np.zeros((dirs.shape[0], K))
    dY = np.zeros((dirs.shape[0], K, 3)) if grad else None
    lib().or_sh_basis(deg, dirs.shape[0], _p(dirs), _p(Y), _p(dY))
    return (Y, dY) if grad else Y


# ---------------------------------------------------------------------------
# loss of the joint optimisation and of the mapping step (L1 parts)
# ---------------------------------------------------------------------------

def loss_and_upstream(cams, render_out, tgt_color, tgt_depth, w_color: float, w_depth: float,
                      mask: Optional[np.ndarray] = None, gate_gamma: Optional[float] = None):
    """Per view v: Lc_v = sum_{p,k} m_p |C - C^| / (3 H W), Ld_v = sum_p m_p
    |D - D^| / (H W).  Total (render part) = (1/V) sum_v (w_c Lc_v + w_d Ld_v).
    The mask m is the optional pixel weight times, if ``gate_gamma`` is given,
    the filter gate of Sec. 3.3: target depth > 0, rendered depth > 0 and
    rendered alpha > gamma (held constant: no gradient through it).
    Returns (Lc [V], Ld [V], dL/dC flat, dL/dD flat); sign(0) = 0."""
    V = len(cams)
    C = render_out["color"]
    D = render_out["depth"]
    A = render_out["alpha"]
    Lc = np.zeros(V)
    Ld = np.zeros(V)
    dC = np.zeros_like(C, dtype=np.float64)
    dD = np.zeros_like(D, dtype=np.float64)
    co = cd = 0
    for v, c in enumerate(cams):
        P = c.width * c.height
        m = np.ones(P) if mask is None else _d(mask[cd:cd + P])
        if gate_gamma is not None:
            g = (_d(tgt_depth[cd:cd + P]) > 0) & (D[cd:cd + P] > 0) & (A[cd:cd + P] > gate_gamma)
            m = m * g
        ec = (C[co:co + 3 * P] - _d(tgt_color[co:co + 3 * P])).reshape(3, P)
        ed = D[cd:cd + P] - _d(tgt_depth[cd:cd + P])
        Lc[v] = float(np.sum(m[None] * np.abs(ec))) / (3 * P)
        Ld[v] = float(np.sum(m * np.abs(ed))) / P
        dC[co:co + 3 * P] = ((w_color / V) / (3 * P) * m[None] * np.sign(ec)).reshape(-1)
        dD[cd:cd + P] = (w_depth / V) / P * m * np.sign(ed)
        co += 3 * P
        cd += P
    return Lc, Ld, dC, dD


# ---------------------------------------------------------------------------
# SSIM term of the mapping loss
# ---------------------------------------------------------------------------
# The paper adds an SSIM loss on the RGB render with weight zeta (Sec. 3.4,
# mapping-loss equation) and does not define it further.  Reading: the usual
# structural similarity with an 11 x 11 Gaussian window of standard deviation
# 1.5 px, constants C1 = 0.01^2 and C2 = 0.03^2 (images in [0, 1]), windows
# clipped at the image border by zero padding (a "same"-size correlation),
# computed per colour channel; L_SSIM of a view = 1 - mean over its pixels and
# channels.

SSIM_RADIUS = 5
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def ssim_window() -> np.ndarray:
    """The 1D window (11 taps, normalised); the 2D window is its outer product."""
    x = np.arange(-SSIM_RADIUS, SSIM_RADIUS + 1, dtype=np.float64)
    g = np.exp(-x * x / (2.0 * SSIM_SIGMA ** 2))
    return g / g.sum()


def _window_mean(img: np.ndarray) -> np.ndarray:
    """Zero-padded same-size correlation of a [H, W] image with the 2D window
    (separable: rows, then columns)."""
    from scipy.ndimage import correlate1d
    g = ssim_window()
    t = correlate1d(img, g, axis=1, mode="constant", cval=0.0)
    return correlate1d(t, g, axis=0, mode="constant", cval=0.0)


def ssim_channel(x: np.ndarray, y: np.ndarray, grad: bool = False):
    """SSIM map of one channel, x rendered and y reference ([H, W]).  With
    ``grad``, also d(sum of the map)/dx.

    Per pixel p: mu_x, mu_y, e_xx, e_yy, e_xy are window means of x, y, x^2,
    y^2, xy; sigma_x^2 = e_xx - mu_x^2, sigma_y^2 = e_yy - mu_y^2,
    sigma_xy = e_xy - mu_x mu_y; s = N / D with
    N = (2 mu_x mu_y + C1)(2 sigma_xy + C2) and
    D = (mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2).
    Reverse mode: s depends on x through mu_x, e_xx and e_xy; with
    A1 = 2 mu_x mu_y + C1, A2 = 2 sigma_xy + C2, B1 = mu_x^2 + mu_y^2 + C1,
    B2 = sigma_x^2 + sigma_y^2 + C2:
    ds/dmu_x = (2 mu_y (A2 - A1) - s 2 mu_x (B2 - B1)) / D,
    ds/de_xx = -s B1 / D, ds/de_xy = 2 A1 / D.  The window mean is a symmetric
    zero-padded correlation, so its transpose is itself: the gradient at q is
    M[ds/dmu_x](q) + 2 x_q M[ds/de_xx](q) + y_q M[ds/de_xy](q)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = _window_mean(x), _window_mean(y)
    exx, eyy, exy = _window_mean(x * x), _window_mean(y * y), _window_mean(x * y)
    sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
    A1 = 2.0 * mx * my + SSIM_C1
    A2 = 2.0 * sxy + SSIM_C2
    B1 = mx * mx + my * my + SSIM_C1
    B2 = sxx + syy + SSIM_C2
    D = B1 * B2
    smap = A1 * A2 / D
    if not grad:
        return smap
    d_mx = (2.0 * my * (A2 - A1) - smap * 2.0 * mx * (B2 - B1)) / D
    d_exx = -smap * B1 / D
    d_exy = 2.0 * A1 / D
    gx = _window_mean(d_mx) + 2.0 * x * _window_mean(d_exx) + y * _window_mean(d_exy)
    return smap, gx


def ssim_views(cams, img, ref, weights=None):
    """Mean SSIM per view of planar colour images concatenated over views
    ([3, H, W] per view, flat), and, with ``weights`` (one per view), the
    gradient of L = sum_v weights[v] (1 - SSIM_v) with respect to ``img``.
    Returns (ssim [V], dL/dimg flat or None)."""
    V = len(cams)
    S = np.zeros(V)
    dimg = None if weights is None else np.zeros(np.asarray(img).shape, np.float64)
    o = 0
    for v, c in enumerate(cams):
        P = c.width * c.height
        X = _d(img[o:o + 3 * P]).reshape(3, c.height, c.width)
        Y = _d(ref[o:o + 3 * P]).reshape(3, c.height, c.width)
        tot = 0.0
        for k in range(3):
            if weights is None:
                sm = ssim_channel(X[k], Y[k])
            else:
                sm, gk = ssim_channel(X[k], Y[k], grad=True)
                dimg[o + k * P:o + (k + 1) * P] = -float(weights[v]) / (3.0 * P) * gk.reshape(-1)
            tot += float(sm.sum())
        S[v] = tot / (3.0 * P)
        o += 3 * P
    return S, dimg


# ---------------------------------------------------------------------------
# Map maintenance: pruning and densification (Sec. 3.4)
# ---------------------------------------------------------------------------
# Readings.  Pruning (Sec. 3.4 pruning equation; the printed cases and the
# text disagree on which side is removed): a Gaussian is removed when its
# opacity o = sigmoid(logit) < tau, the order of the others is kept.
# Densification: every pixel of a view whose rendered alpha (the border mask
# M_b) is <= gamma -- every pixel on the first frame -- and whose target depth
# d is > 0 gets one new Gaussian: its mean back-projects the pixel's sample
# point (x, y) to depth d, it is isotropic with radius d / fx (a one-pixel
# footprint, Eq. d read as r = d / f), identity rotation, opacity 1/2 (logit
# 0; the paper gives no initial value), and the target colour (with SH, the
# DC coefficient reproduces it and the others are 0).  New Gaussians follow
# the existing ones, in view order, then row-major pixel order.

SH_C0 = 0.28209479177387814   # Y_00 of the real orthonormal basis


def prune(params: Dict[str, np.ndarray], tau: float):
    """params: dict of arrays with the Gaussian index first.  Returns (kept
    params, kept indices)."""
    opl = _d(params["opacity_logits"]).reshape(-1)
    o = 1.0 / (1.0 + np.exp(-opl))
    keep = np.nonzero(~(o < tau))[0]
    return {k: np.asarray(v)[keep] for k, v in params.items()}, keep


def densify(cams, poses, alpha, tgt_color, tgt_depth, gamma: float, all_pixels: bool, sh_degree: int = -1,
            isotropic: bool = False):
    """New Gaussians (dict of FP64 arrays: means [m,3], log_scales [m,3],
    quats [m,4], opacity_logits [m], colors [m,3] or [m,K,3]; isotropic:
    log_radius [m] in place of log_scales and quats) and, for each, its
    (view, x, y)."""
    K = 1 if sh_degree < 0 else (sh_degree + 1) ** 2
    means, ls, cols, where = [], [], [], []
    po = 0
    for v, c in enumerate(cams):
        P = c.width * c.height
        A = _d(alpha[po:po + P]).reshape(c.height, c.width)
        Dt = _d(tgt_depth[po:po + P]).reshape(c.height, c.width)
        Ct = _d(tgt_color[3 * po:3 * po + 3 * P]).reshape(3, c.height, c.width)
        T = _d(poses[v]).reshape(4, 4)
        R, t = T[:3, :3], T[:3, 3]
        for y in range(c.height):
            for x in range(c.width):
                d = Dt[y, x]
                if not (d > 0.0) or not (all_pixels or A[y, x] <= gamma):
                    continue
                pc = np.array([(x - c.cx) / c.fx * d, (y - c.cy) / c.fy * d, d])
                means.append(R.T @ (pc - t))
                ls.append(np.full(3, np.log(d / c.fx)))
                cols.append(Ct[:, y, x])
                where.append((v, x, y))
        po += P
    m = len(means)
    if isotropic:
        out = {"means": np.array(means).reshape(m, 3), "log_radius": np.array(ls).reshape(m, 3)[:, 0],
               "opacity_logits": np.zeros(m)}
    else:
        out = {"means": np.array(means).reshape(m, 3), "log_scales": np.array(ls).reshape(m, 3),
               "quats": np.tile([1.0, 0.0, 0.0, 0.0], (m, 1)), "opacity_logits": np.zeros(m)}
    rgb = np.array(cols).reshape(m, 3)
    if sh_degree < 0:
        out["colors"] = rgb
    else:
        sh = np.zeros((m, K, 3))
        sh[:, 0, :] = (rgb - 0.5) / SH_C0
        out["colors"] = sh
    return out, np.array(where, np.int64).reshape(m, 3)


def adam_groups(n: int, sh_degree: int, V: int, isotropic: bool = False):
    """(offset, per-Gaussian width) of each parameter group in the Adam
    moment layout (means, log-scales or log-radius, quaternions, opacity
    logits, colours), and the offset of the 6V pose moments."""
    K = 1 if sh_degree < 0 else (sh_degree + 1) ** 2
    widths = [3, 1, 0, 1, 3 * K] if isotropic else [3, 3, 4, 1, 3 * K]
    offs, o = [], 0
    for w in widths:
        offs.append(o)
        o += w * n
    return list(zip(offs, widths)), o


def adam_relayout(m: np.ndarray, n: int, sh_degree: int, V: int, src_index: np.ndarray, n_new: int,
                  isotropic: bool = False):
    """Moments of n_new Gaussians whose i-th comes from old Gaussian
    src_index[i] (or is new with zero moments when src_index[i] < 0); the pose
    moments are carried over."""
    old, pose_old = adam_groups(n, sh_degree, V, isotropic)
    new, pose_new = adam_groups(n_new, sh_degree, V, isotropic)
    out = np.zeros(pose_new + 6 * V)
    for (oo, w), (on, _) in zip(old, new):
        src = np.asarray(m[oo:oo + w * n]).reshape(n, w)
        dst = out[on:on + w * n_new].reshape(n_new, w)
        ok = src_index >= 0
        dst[ok] = src[src_index[ok]]
    out[pose_new:] = m[pose_old:pose_old + 6 * V]
    return out


# ---------------------------------------------------------------------------
# SE(3) and Adam
# ---------------------------------------------------------------------------

def hat(w) -> np.ndarray:
    w = np.asarray(w, np.float64)
    return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])


def se3_exp(xi) -> np.ndarray:
    """Closed-form exponential of the twist xi = (v, w): rotation by Rodrigues'
    formula, translation V(w) v."""
    xi = np.asarray(xi, np.float64)
    v, w = xi[:3], xi[3:]
    th = float(np.linalg.norm(w))
    Wm = hat(w)
    if th < 1e-8:
        R = np.eye(3) + Wm + 0.5 * Wm @ Wm
        Vm = np.eye(3) + 0.5 * Wm + Wm @ Wm / 6.0
    else:
        a = np.sin(th) / th
        b = (1 - np.cos(th)) / th ** 2
        c = (th - np.sin(th)) / th ** 3
        R = np.eye(3) + a * Wm + b * Wm @ Wm
        Vm = np.eye(3) + b * Wm + c * Wm @ Wm
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = Vm @ v
    return T


def se3_left_jacobian(xi, terms: int = 60) -> np.ndarray:
    """Left Jacobian J_l of SE(3) at the twist xi = (v, w): the 6x6 matrix with
    Exp(xi + e) = Exp(J_l e) Exp(xi) to first order in e, from its defining
    series sum_n ad(xi)^n / (n + 1)!, ad(xi) = [[w^, v^], [0, w^]] (the
    bracket of se(3) in (v, w) coordinates).  The gradient of L(Exp(xi) T)
    with respect to xi is J_l(xi)^T times the left-perturbation gradient at
    Exp(xi) T (the pose tangent of the joint optimisation, Sec. 3.3)."""
    xi = np.asarray(xi, np.float64)
    ad = np.zeros((6, 6))
    ad[:3, :3] = hat(xi[3:])
    ad[:3, 3:] = hat(xi[:3])
    ad[3:, 3:] = hat(xi[3:])
    J = np.eye(6)
    term = np.eye(6)
    for n in range(1, terms):
        term = term @ ad / (n + 1)
        J = J + term
    return J


def adam_step(param, grad, m, v, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), t = index of this update starting at 1.
    Returns (delta, m, v) with delta the step to ADD to the parameter."""
    grad = _d(grad)
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return -lr * mh / (np.sqrt(vh) + eps), m, v
