"""Seeded synthetic scenes for the Gaussian-splatting hot path.

This module only draws inputs: Gaussian parameters, cameras, poses, targets
and 2D-3D matches.  It holds none of the renderer's arithmetic (no
projection of Gaussians, no compositing, no loss), so the FP64 oracle and the
HIP path can both consume its output without sharing any method code.

The paper's workload (TUM RGB-D sequences, Sec. 4.1) is not available; the
scenes below stand in for it with the shapes and value distributions of five
fixed configurations:

* ``c1`` - 2,000 Gaussians, one 64x48 view, f=60, identity pose.
* ``c2`` - 200,000 Gaussians in a 4x4x4 m box in front of one 640x480 view,
  f=525, estimated pose perturbed by 0.02 rad / 0.05 m.
* ``c3`` - 1,000,000 Gaussians in an 8x8x3 m room shell (70 % on the six
  planes, 30 % in the volume), 8 views at 1200x680, f=600, smooth trajectory.
* ``c4`` - 2,000,000 Gaussians in the room, 4-16 views of uneven resolution
  and visible count, plus 1,000-2,000 ORB-style 2D-3D matches per view with
  1 px noise and 5 % outliers (for the Huber re-projection term).
* ``c5`` - 3,000,000 Gaussians with SH degree 3 colour, 16 views at 1200x680
  from a sliding window on a 515-pose trajectory.

Every config accepts size overrides so tests can build the same scene shape
at a size the oracle finishes in seconds.

Camera convention: OpenCV (x right, y down, z forward).  ``T_cw`` is the
4x4 world-to-camera transform, row-major.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

F32 = np.float32


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    def as_tuple(self):
        return (self.width, self.height, self.fx, self.fy, self.cx, self.cy)

    @property
    def npix(self) -> int:
        return self.width * self.height


@dataclass
class Scene:
    name: str
    means: np.ndarray            # [N,3] f32
    log_scales: np.ndarray       # [N,3] f32
    quats: np.ndarray            # [N,4] f32, (w, x, y, z)
    opacity_logits: np.ndarray   # [N] f32
    colors: np.ndarray           # [N,3] (RGB) or [N,K,3] (SH) f32
    sh_degree: int               # -1 = RGB
    cams: List[Camera]
    poses: np.ndarray            # [V,4,4] f32 estimated world->camera (optimised)
    poses_true: np.ndarray       # [V,4,4] f32 true world->camera (targets rendered here)
    w_color: float = 1.0
    w_depth: float = 0.0
    w_reproj: float = 0.0
    huber_delta: float = 2.0
    target_color: Optional[np.ndarray] = None   # flat [sum 3HW] f32 when given by the config
    target_depth: Optional[np.ndarray] = None   # flat [sum HW] f32
    points: Optional[np.ndarray] = None         # [M,3] f32
    uv: Optional[np.ndarray] = None             # [M,2] f32
    view_idx: Optional[np.ndarray] = None       # [M] int32
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def V(self) -> int:
        return len(self.cams)

    @property
    def npix(self) -> int:
        return sum(c.npix for c in self.cams)

    def pix_offsets(self) -> np.ndarray:
        off = np.zeros(self.V + 1, dtype=np.int64)
        for i, c in enumerate(self.cams):
            off[i + 1] = off[i] + c.npix
        return off

    @property
    def isotropic(self) -> bool:
        """The paper's eight-parameter Gaussian: log_scales [N,1] holds one
        log radius per Gaussian and quats is empty [N,0]."""
        return bool(self.extra.get("isotropic", False))

    def subset_views(self, idx) -> "Scene":
        """Same Gaussians, only the views in ``idx`` (matches are dropped)."""
        idx = list(idx)
        s = Scene(self.name, self.means, self.log_scales, self.quats, self.opacity_logits,
                  self.colors, self.sh_degree, [self.cams[i] for i in idx],
                  self.poses[idx].copy(), self.poses_true[idx].copy(), self.w_color,
                  self.w_depth, self.w_reproj, self.huber_delta, extra=dict(self.extra))
        return s


# ---------------------------------------------------------------------------
# small geometry helpers (generic rigid-body algebra, not the renderer)
# ---------------------------------------------------------------------------

def _rotvec_to_matrix(rv: np.ndarray) -> np.ndarray:
    from scipy.spatial.transform import Rotation
    return Rotation.from_rotvec(np.asarray(rv, dtype=np.float64)).as_matrix()


def _unit(rng: np.random.Generator, k: int = 3) -> np.ndarray:
    v = rng.standard_normal(k)
    return v / np.linalg.norm(v)


def look_pose(centre: np.ndarray, forward: np.ndarray, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """World->camera 4x4 for a camera at ``centre`` looking along ``forward``.

    Camera axes (OpenCV): x right, y down, z forward; ``up`` is the world up.
    """
    f = np.asarray(forward, np.float64)
    f = f / np.linalg.norm(f)
    u = np.asarray(up, np.float64)
    right = np.cross(f, u)
    if np.linalg.norm(right) < 1e-8:
        right = np.cross(f, np.array([1.0, 0.0, 0.0]))
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    R_wc = np.stack([right, down, f], axis=1)   # columns = camera axes in world
    R_cw = R_wc.T
    T = np.eye(4)
    T[:3, :3] = R_cw
    T[:3, 3] = -R_cw @ np.asarray(centre, np.float64)
    return T


def perturb_pose(T_cw: np.ndarray, rng: np.random.Generator, rot=0.02, trans=0.05) -> np.ndarray:
    """Left-multiply a rigid motion of ``rot`` rad about a random axis and a
    translation of ``trans`` m along a random direction."""
    a = _unit(rng)
    b = _unit(rng)
    D = np.eye(4)
    D[:3, :3] = _rotvec_to_matrix(rot * a)
    D[:3, 3] = trans * b
    return D @ T_cw


# ---------------------------------------------------------------------------
# Gaussian parameter draws (fixed order: means, log-scales, quats, opacity
# logits, colours)
# ---------------------------------------------------------------------------

def _draw_params(rng: np.random.Generator, means: np.ndarray, sh_degree: int = -1):
    n = means.shape[0]
    log_scales = rng.normal(-3.0, 0.5, size=(n, 3))
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opl = rng.standard_normal(n)
    if sh_degree < 0:
        colors = rng.uniform(0.0, 1.0, size=(n, 3))
    else:
        K = (sh_degree + 1) ** 2
        colors = rng.normal(0.0, 0.1, size=(n, K, 3))
        colors[:, 0, :] = rng.uniform(0.0, 1.0, size=(n, 3))
    return (means.astype(F32), log_scales.astype(F32), q.astype(F32), opl.astype(F32),
            colors.astype(F32))


def _box_means(rng, n, xy=1.0, z=(1.0, 5.0)):
    m = np.empty((n, 3))
    m[:, 0] = rng.uniform(-xy, xy, n)
    m[:, 1] = rng.uniform(-xy, xy, n)
    m[:, 2] = rng.uniform(z[0], z[1], n)
    return m


ROOM_LO = np.array([-4.0, -4.0, 0.0])
ROOM_HI = np.array([4.0, 4.0, 3.0])


def room_means(rng: np.random.Generator, n: int, lo=ROOM_LO, hi=ROOM_HI, shell=0.7) -> np.ndarray:
    """``shell`` of the points on the six planes of the box (area-proportional),
    the rest uniform in the volume."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    ext = hi - lo
    n_shell = int(round(shell * n))
    n_vol = n - n_shell
    # plane k: axis a = k // 2, side = k % 2; its area is the product of the other two extents
    areas = np.array([ext[(a + 1) % 3] * ext[(a + 2) % 3] for a in (0, 0, 1, 1, 2, 2)])
    plane = rng.choice(6, size=n_shell, p=areas / areas.sum())
    pts = lo + rng.uniform(0.0, 1.0, size=(n_shell, 3)) * ext
    axis = plane // 2
    side = plane % 2
    pts[np.arange(n_shell), axis] = np.where(side == 0, lo[axis], hi[axis])
    vol = lo + rng.uniform(0.0, 1.0, size=(n_vol, 3)) * ext
    m = np.concatenate([pts, vol], axis=0)
    return m[rng.permutation(n)]


def _circle_trajectory(rng: np.random.Generator, n_poses: int, radius=1.5, height=1.5,
                       step=0.15, wobble=0.1) -> np.ndarray:
    """Cameras on a horizontal circle, looking outward, with a smooth seeded
    yaw/pitch wobble below ``wobble`` rad."""
    phase = rng.uniform(0, 2 * np.pi, size=4)
    poses = []
    for k in range(n_poses):
        th = k * step
        c = np.array([radius * np.cos(th), radius * np.sin(th), height])
        yaw = th + wobble * 0.9 * np.sin(0.37 * k + phase[0])
        pitch = wobble * 0.9 * np.sin(0.23 * k + phase[1])
        f = np.array([np.cos(yaw) * np.cos(pitch), np.sin(yaw) * np.cos(pitch), np.sin(pitch)])
        poses.append(look_pose(c, f))
    return np.stack(poses)


def _scaled_cam(w, h, f, width=None, height=None) -> Camera:
    """Camera of size (width, height) with the focal length scaled so the
    field of view of the (w, h, f) camera is kept; principal point at the
    centre."""
    W = int(width or w)
    H = int(height or h)
    s = W / w
    return Camera(W, H, f * s, f * s, W / 2.0, H / 2.0)


# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------

def c1(n: int = 2000, width: int = 64, height: int = 48, seed: int = 1) -> Scene:
    rng = np.random.Generator(np.random.PCG64(seed))
    means = _box_means(rng, n, 1.0)
    p = _draw_params(rng, means)
    s = width / 64.0
    cam = Camera(width, height, 60.0 * s, 60.0 * s, 32.0 * s, 24.0 * s)
    T = np.eye(4)[None]
    tgt = rng.uniform(0.0, 1.0, size=3 * width * height).astype(F32)
    return Scene("c1", *p, -1, [cam], T.astype(F32), T.astype(F32), 1.0, 0.0, 0.0, 2.0,
                 target_color=tgt, target_depth=np.zeros(width * height, F32))


def c2(n: int = 200_000, width: int = 640, height: int = 480, seed: int = 2) -> Scene:
    rng = np.random.Generator(np.random.PCG64(seed))
    means = _box_means(rng, n, 2.0)
    p = _draw_params(rng, means)
    cam = _scaled_cam(640, 480, 525.0, width, height)
    T_true = np.eye(4)
    T_est = perturb_pose(T_true, rng)
    return Scene("c2", *p, -1, [cam], T_est[None].astype(F32), T_true[None].astype(F32),
                 1.0, 0.1, 0.0, 2.0)


def c3(n: int = 1_000_000, views: int = 8, width: int = 1200, height: int = 680,
       seed: int = 3) -> Scene:
    rng = np.random.Generator(np.random.PCG64(seed))
    means = room_means(rng, n)
    p = _draw_params(rng, means)
    cam = _scaled_cam(1200, 680, 600.0, width, height)
    T_true = _circle_trajectory(rng, views)
    T_est = np.stack([perturb_pose(T, rng) for T in T_true])
    return Scene("c3", *p, -1, [cam] * views, T_est.astype(F32), T_true.astype(F32),
                 1.0, 0.1, 0.0, 2.0)


C4_RES = ((320, 240, 262.5), (640, 480, 525.0), (1200, 680, 600.0))


def _visible_fraction_proxy(means_sub: np.ndarray, T_cw: np.ndarray, cam: Camera) -> float:
    """Fraction of points in front of the camera and inside its view cone;
    used only to place cameras."""
    pc = means_sub @ T_cw[:3, :3].T + T_cw[:3, 3]
    z = pc[:, 2]
    ok = z > 0.2
    hx = cam.width / (2 * cam.fx)
    hy = cam.height / (2 * cam.fy)
    zz = np.where(ok, z, 1.0)
    ok &= (np.abs(pc[:, 0] / zz) < hx) & (np.abs(pc[:, 1] / zz) < hy)
    return float(ok.mean())


def c4(n: int = 2_000_000, step: int = 0, res_scale: float = 1.0, vis_range=(50_000, 2_000_000),
       views: Optional[int] = None, matches=(1000, 2000), seed: int = 4) -> Scene:
    rng_scene = np.random.Generator(np.random.PCG64(seed))
    means = room_means(rng_scene, n)
    p = _draw_params(rng_scene, means)
    rng = np.random.Generator(np.random.PCG64(4000 + step if seed == 4 else seed * 1000 + step))
    V = int(views) if views is not None else int(rng.integers(4, 17))
    sub = means[rng.choice(n, size=min(n, 20_000), replace=False)]
    cams, Ts = [], []
    lo_v, hi_v = vis_range
    for _ in range(V):
        w, h, f = C4_RES[int(rng.integers(0, 3))]
        W = max(16, int(round(w * res_scale)))
        H = max(16, int(round(h * res_scale)))
        cam = Camera(W, H, f * W / w, f * W / w, W / 2.0, H / 2.0)
        target = np.exp(rng.uniform(np.log(lo_v), np.log(hi_v))) / 2_000_000.0
        best = None
        for _try in range(200):
            # camera anywhere from inside the room to 6 m outside it, aimed near the centre
            c = rng.uniform(ROOM_LO - 6.0, ROOM_HI + 6.0)
            c[2] = rng.uniform(0.3, 2.7)
            aim = np.array([0.0, 0.0, 1.5]) + rng.normal(0.0, 1.5, 3)
            fwd = aim - c
            if np.linalg.norm(fwd) < 0.5:
                continue
            T = look_pose(c, fwd)
            frac = _visible_fraction_proxy(sub, T, cam)
            err = abs(frac - target) / target
            if best is None or err < best[0]:
                best = (err, T)
            if err <= 0.1:
                break
        cams.append(cam)
        Ts.append(best[1])
    T_true = np.stack(Ts)
    T_est = np.stack([perturb_pose(T, rng) for T in T_true])
    # ORB-style matches: a pixel and a depth are drawn, the 3D point is its
    # back-projection under the true pose; the observation gets 1 px noise and
    # 5 % are replaced by uniform pixels (outliers).
    pts, uvs, vidx = [], [], []
    for v in range(V):
        cam = cams[v]
        M = int(rng.integers(matches[0], matches[1] + 1))
        px = rng.uniform(0, cam.width - 1, M)
        py = rng.uniform(0, cam.height - 1, M)
        z = rng.uniform(1.0, 6.0, M)
        xc = np.stack([(px - cam.cx) / cam.fx * z, (py - cam.cy) / cam.fy * z, z], axis=1)
        R_cw = T_true[v][:3, :3]
        t_cw = T_true[v][:3, 3]
        Pw = (xc - t_cw) @ R_cw          # = R_cw^T (xc - t)
        obs = np.stack([px, py], axis=1) + rng.normal(0.0, 1.0, (M, 2))
        out = rng.uniform(0.0, 1.0, M) < 0.05
        obs[out, 0] = rng.uniform(0, cam.width - 1, out.sum())
        obs[out, 1] = rng.uniform(0, cam.height - 1, out.sum())
        pts.append(Pw)
        uvs.append(obs)
        vidx.append(np.full(M, v, np.int32))
    return Scene("c4", *p, -1, cams, T_est.astype(F32), T_true.astype(F32), 1.0, 0.1, 0.5, 2.0,
                 points=np.concatenate(pts).astype(F32), uv=np.concatenate(uvs).astype(F32),
                 view_idx=np.concatenate(vidx).astype(np.int32))


def c5(n: int = 3_000_000, views: int = 16, width: int = 1200, height: int = 680, window: int = 0,
       traj_len: int = 515, seed: int = 5) -> Scene:
    rng = np.random.Generator(np.random.PCG64(seed))
    means = room_means(rng, n)
    p = _draw_params(rng, means, sh_degree=3)
    cam = _scaled_cam(1200, 680, 600.0, width, height)
    traj = _circle_trajectory(rng, traj_len, step=0.05)
    T_true = traj[window:window + views]
    # the estimated poses the mapping holds fixed: perturbed as in c2, so the
    # rendering loss against the true-pose targets is not zero
    T_est = np.stack([perturb_pose(T, rng) for T in T_true])
    return Scene("c5", *p, 3, [cam] * views, T_est.astype(F32), T_true.astype(F32),
                 1.0, 0.1, 0.0, 2.0, extra={"window": window, "trajectory": traj.astype(F32)})


def isotropic(s: Scene) -> Scene:
    """The same scene with the paper's own Gaussian (Sec. 3.4): one radius per
    Gaussian instead of three scales and a rotation.  The log radius is the
    first log-scale draw (the same N(-3, 0.5) distribution); quats becomes an
    empty [N,0] array."""
    extra = dict(s.extra)
    extra["isotropic"] = True
    return Scene(s.name + "_iso", s.means, np.ascontiguousarray(s.log_scales[:, :1]),
                 np.zeros((s.n, 0), F32), s.opacity_logits, s.colors, s.sh_degree, s.cams, s.poses,
                 s.poses_true, s.w_color, s.w_depth, s.w_reproj, s.huber_delta, s.target_color,
                 s.target_depth, s.points, s.uv, s.view_idx, extra)


CONFIGS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5}


def random_cotangents(scene: Scene, seed: int, scale: float = 1e-3) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Random upstream gradients (dC, dD, dA) for driving a backward pass."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = scene.npix
    dC = (rng.standard_normal(3 * P) * scale).astype(F32)
    dD = (rng.standard_normal(P) * scale).astype(F32)
    dA = (rng.standard_normal(P) * scale).astype(F32)
    return dC, dD, dA


def sample_pixels(cam: Camera, k: int, seed: int) -> np.ndarray:
    """``k`` distinct pixel coordinates (x, y) of one view, int32 [k,2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = min(k, cam.npix)
    flat = rng.choice(cam.npix, size=k, replace=False)
    flat.sort()
    return np.stack([flat % cam.width, flat // cam.width], axis=1).astype(np.int32)


def synthetic_binning_records(sizes: List[Tuple[int, int]], n: int, seed: int, empty_frac=0.2,
                              tie_frac=0.3, max_ext=96):
    """Random per-record pixel rects and FP32 depths for the binning stage.

    ``sizes`` holds (width, height) per view; record ``v*n + i`` belongs to
    view ``v``.  Returns ``rect`` u32 [V*n,2] packed as (x0 | x1<<16,
    y0 | y1<<16) with inclusive bounds inside the image and an empty rect
    encoded as x0 > x1, and ``depth`` f32 [V*n] (positive).  A share of the
    depths is drawn from a small pool so that equal keys occur.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    V = len(sizes)
    rect = np.zeros((V * n, 2), np.uint32)
    depth = rng.uniform(0.2, 30.0, V * n).astype(F32)
    pool = rng.uniform(0.2, 30.0, 7).astype(F32)
    ties = rng.uniform(0, 1, V * n) < tie_frac
    depth[ties] = pool[rng.integers(0, 7, ties.sum())]
    for v, (W, H) in enumerate(sizes):
        x0 = rng.integers(0, W, n)
        y0 = rng.integers(0, H, n)
        x1 = np.minimum(W - 1, x0 + rng.integers(0, max_ext, n))
        y1 = np.minimum(H - 1, y0 + rng.integers(0, max_ext, n))
        empty = rng.uniform(0, 1, n) < empty_frac
        x0 = np.where(empty, 1, x0)
        x1 = np.where(empty, 0, x1)
        rect[v * n:(v + 1) * n, 0] = (x0 | (x1 << 16)).astype(np.uint32)
        rect[v * n:(v + 1) * n, 1] = (y0 | (y1 << 16)).astype(np.uint32)
    return rect, depth
