"""Python binding of the C ABI (include/gs.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of libgs.so.  PyTorch provides device memory and the current stream.
There is no CPU fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import _abi as A


class GSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{A.STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t: Optional[torch.Tensor], numel: int, name: str, dtype=torch.float32, device=None):
    """Host-side check that a device buffer matches what the kernels index."""
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


def _check_gaussians(g: "Gaussians", device):
    n = g.n
    _need(g.means, 3 * n, "means", device=device)
    _need(g.log_scales, n if g.isotropic else 3 * n, "log_scales", device=device)
    _need(g.quats, 0 if g.isotropic else 4 * n, "quats", device=device)
    _need(g.opacity_logits, n, "opacity_logits", device=device)
    _need(g.colors, 3 * n * sh_coeffs(g.sh_degree), "colors", device=device)


def _dev_f32(t, device) -> torch.Tensor:
    t = torch.as_tensor(t, dtype=torch.float32, device=device)
    return t.contiguous()


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    @property
    def npix(self) -> int:
        return self.width * self.height


def as_cameras(cams) -> List[Camera]:
    out = []
    for c in cams:
        if isinstance(c, Camera):
            out.append(c)
        elif hasattr(c, "as_tuple"):
            out.append(Camera(*c.as_tuple()))
        else:
            out.append(Camera(*c))
    return out


def cam_array(cams: Sequence[Camera]):
    arr = (A.gs_camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = A.gs_camera(int(c.width), int(c.height), float(c.fx), float(c.fy), float(c.cx), float(c.cy))
    return arr


def sh_coeffs(sh_degree: int) -> int:
    return 1 if sh_degree < 0 else (sh_degree + 1) ** 2


def floats_per_gaussian(sh_degree: int, isotropic: bool = False) -> int:
    """FP32 values per Gaussian in the parameter and Adam moment layouts:
    means 3, log-scales 3 (log radius 1), quaternion 4 (none), opacity 1,
    colour 3K -- 14 anisotropic, the paper's 8 isotropic, with RGB."""
    return (5 if isotropic else 11) + 3 * sh_coeffs(sh_degree)


@dataclass
class Gaussians:
    """Device FP32 parameters (structure of arrays).  isotropic: the paper's
    eight-parameter Gaussian, log_scales [n,1] holds the log radius and
    quats is empty [n,0]."""
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    opacity_logits: torch.Tensor
    colors: torch.Tensor
    sh_degree: int = -1
    isotropic: bool = False

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @classmethod
    def from_arrays(cls, means, log_scales, quats, opacity_logits, colors, sh_degree=-1, device="cuda",
                    isotropic=False):
        m = _dev_f32(means, device).reshape(-1, 3)
        if isotropic:
            ls = _dev_f32(log_scales, device).reshape(-1, 1)
            q = torch.empty((m.shape[0], 0), dtype=torch.float32, device=device)
        else:
            ls = _dev_f32(log_scales, device).reshape(-1, 3)
            q = _dev_f32(quats, device).reshape(-1, 4)
        return cls(m, ls, q, _dev_f32(opacity_logits, device).reshape(-1), _dev_f32(colors, device),
                   int(sh_degree), bool(isotropic))

    @classmethod
    def isotropic_from_arrays(cls, means, log_radius, opacity_logits, colors, sh_degree=-1, device="cuda"):
        """The paper's Gaussian: centre, one log radius, opacity logit, colour."""
        return cls.from_arrays(means, log_radius, None, opacity_logits, colors, sh_degree, device, True)

    @classmethod
    def from_scene(cls, s, device="cuda"):
        return cls.from_arrays(s.means, s.log_scales, s.quats, s.opacity_logits, s.colors, s.sh_degree, device,
                               bool(getattr(s, "isotropic", False)))

    def like(self, *tensors) -> "Gaussians":
        """Another set of this layout (sh_degree, isotropic) from five tensors."""
        return Gaussians(*tensors, self.sh_degree, self.isotropic)

    def struct(self) -> A.gs_gaussians:
        return A.gs_gaussians(self.n, self.sh_degree, int(self.isotropic), _p(self.means), _p(self.log_scales),
                              _p(self.quats) if not self.isotropic else None, _p(self.opacity_logits),
                              _p(self.colors))

    def zeros_like(self) -> "Gaussians":
        return self.like(*(torch.zeros_like(t) for t in self.tensors()))

    @property
    def floats_per_gaussian(self) -> int:
        return floats_per_gaussian(self.sh_degree, self.isotropic)

    def grad_struct(self) -> A.gs_gaussian_grads:
        return A.gs_gaussian_grads(_p(self.means), _p(self.log_scales), None if self.isotropic else _p(self.quats),
                                   _p(self.opacity_logits), _p(self.colors))

    def tensors(self) -> Tuple[torch.Tensor, ...]:
        return (self.means, self.log_scales, self.quats, self.opacity_logits, self.colors)


def split_images(cams: Sequence[Camera], color: torch.Tensor, depth: torch.Tensor, alpha: torch.Tensor):
    """Per-view [3,H,W], [H,W], [H,W] views of the concatenated outputs."""
    out = []
    o = 0
    for c in cams:
        P = c.npix
        out.append((color[3 * o:3 * (o + P)].view(3, c.height, c.width), depth[o:o + P].view(c.height, c.width),
                    alpha[o:o + P].view(c.height, c.width)))
        o += P
    return out


class Context:
    """One library context (one device; use one per stream)."""

    def __init__(self, device: Optional[int] = None):
        self.lib = A.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP path has no CPU fallback")
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = ctypes.c_void_p()
        rc = self.lib.gs_create(ctypes.byref(h), self.device)
        if rc != 0:
            raise GSError(rc, self.lib.gs_last_error(None).decode())
        self.h = h
        self.pair_estimate = 1 << 16
        self.bin_choice = (64, 64)
        self.bwd_tile_choice = (0, 0)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.gs_destroy(h)
            self.h = None

    def _check(self, rc: int):
        if rc != 0:
            raise GSError(rc, self.lib.gs_last_error(self.h).decode())

    @property
    def torch_device(self):
        return torch.device("cuda", self.device)

    # -------------------------------------------------------------- sizes
    def state_bytes(self, cams, n: int, capacity: int, bin=(0, 0)) -> int:
        cams = as_cameras(cams)
        b = self.lib.gs_state_bytes(cam_array(cams), len(cams), n, capacity, bin[0], bin[1])
        if b == 0:
            raise GSError(A.GS_EINVAL, "invalid arguments for gs_state_bytes")
        return int(b)

    def workspace_bytes(self, cams, n: int, sh_degree: int, capacity: int, bin=(0, 0)) -> int:
        cams = as_cameras(cams)
        b = self.lib.gs_step_workspace_bytes(cam_array(cams), len(cams), n, sh_degree, capacity, bin[0], bin[1])
        if b == 0:
            raise GSError(A.GS_EINVAL, "invalid arguments for gs_step_workspace_bytes")
        return int(b)

    def set_tile(self, tw: int, th: int, ppt: Optional[int] = None):
        self._check(self.lib.gs_set_tile(self.h, tw, th))
        if ppt is not None:
            self._check(self.lib.gs_set_pixels_per_thread(self.h, tw, th, ppt))

    def ppt_choice(self, tile, backward: bool = False) -> int:
        """Pixels per thread the compositing kernels use for ``tile`` (tw, th)."""
        r = int(self.lib.gs_get_pixels_per_thread(self.h, int(backward), int(tile[0]), int(tile[1])))
        if r < 0:
            self._check(r)
        return r

    def set_bwd_shape(self, tw: int, th: int, ppt: int):
        """The backward's own tile and pixels per thread (0, 0, 0: the forward's)."""
        self._check(self.lib.gs_set_bwd_shape(self.h, tw, th, ppt))
        self.bwd_tile_choice = (int(tw), int(th))

    def set_bin(self, bw: int, bh: int):
        self._check(self.lib.gs_set_bin(self.h, bw, bh))
        self.bin_choice = (int(bw), int(bh)) if (bw, bh) != (0, 0) else (64, 64)

    # -------------------------------------------------------------- render
    def forward(self, g: Gaussians, cams, poses: torch.Tensor, tile=(0, 0), capacity: Optional[int] = None,
                bin=(0, 0), sync: bool = True):
        """Returns (color, depth, alpha, state, plan).  sync=False: no host
        synchronisation (gs_render_forward_async) with ``capacity`` pairs (the
        context's estimate by default); an overflow gives an empty render,
        flagged in the state (``state_status``)."""
        cams = as_cameras(cams)
        ca = cam_array(cams)
        V = len(cams)
        npix = sum(c.npix for c in cams)
        dev = self.torch_device
        color = torch.empty(3 * npix, dtype=torch.float32, device=dev)
        depth = torch.empty(npix, dtype=torch.float32, device=dev)
        alpha = torch.empty(npix, dtype=torch.float32, device=dev)
        poses = poses.contiguous()
        _check_gaussians(g, dev)
        _need(poses, 16 * V, "poses", device=dev)
        cap = int(capacity if capacity is not None else self.pair_estimate)
        gst = g.struct()
        bw, bh = self._bin(bin)
        if not sync:
            nbytes = self.state_bytes(cams, g.n, cap, (bw, bh))
            state = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            plan = A.gs_plan(tile[0], tile[1], bw, bh, cap, 0, 0)
            self._check(self.lib.gs_render_forward_async(self.h, ctypes.byref(gst), ca, _p(poses), V, _p(color),
                                                         _p(depth), _p(alpha), _p(state), nbytes,
                                                         ctypes.byref(plan), _stream()))
            return color, depth, alpha, state, plan
        for _ in range(3):
            nbytes = self.state_bytes(cams, g.n, cap, (bw, bh))
            state = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            plan = A.gs_plan(tile[0], tile[1], bw, bh, cap, 0, 0)
            rc = self.lib.gs_render_forward(self.h, ctypes.byref(gst), ca, _p(poses), V, _p(color), _p(depth),
                                            _p(alpha), _p(state), nbytes, ctypes.byref(plan), _stream())
            if rc == A.GS_ECAPACITY:
                cap = int(plan.n_pairs * 1.25) + 1024
                self.pair_estimate = max(self.pair_estimate, cap)
                continue
            self._check(rc)
            self.pair_estimate = max(self.pair_estimate, int(plan.n_pairs * 1.25) + 1024)
            return color, depth, alpha, state, plan
        raise GSError(A.GS_ECAPACITY, "pair capacity did not converge")

    def state_status(self, state: torch.Tensor) -> Dict[str, int]:
        """Flags and counts of the pass that wrote ``state`` (a forward state
        or a mapping-step workspace); synchronises the stream."""
        f = ctypes.c_int32()
        npairs = ctypes.c_int64()
        nvis = ctypes.c_int64()
        self._check(self.lib.gs_step_status(self.h, _p(state), state.numel(), ctypes.byref(f), ctypes.byref(npairs),
                                            ctypes.byref(nvis), _stream()))
        return {"flags": int(f.value), "n_pairs": int(npairs.value), "n_visible": int(nvis.value)}

    def check_async(self) -> Dict[str, int]:
        """state_status of the last render(..., sync=False), raising GSError
        when it overflowed its capacity (or read a non-finite parameter)."""
        st = getattr(self, "last_async_state", None)
        if st is None:
            return {"flags": 0, "n_pairs": 0, "n_visible": 0}
        s = self.state_status(st)
        if s["flags"] & 1:
            self.pair_estimate = max(self.pair_estimate, int(s["n_pairs"] * 1.25) + 1024)
            raise GSError(A.GS_ECAPACITY, f"an asynchronous render needed {s['n_pairs']} pairs")
        if s["flags"] & 4:
            raise GSError(A.GS_EINVAL, "an asynchronous render read a non-finite Gaussian parameter")
        if s["flags"]:
            raise GSError(A.GS_EDEVICE, f"asynchronous render flags {s['flags']}")
        return s

    def backward(self, g: Gaussians, cams, poses: torch.Tensor, state: torch.Tensor, plan, dC=None, dD=None,
                 dA=None) -> Tuple[Gaussians, torch.Tensor]:
        cams = as_cameras(cams)
        V = len(cams)
        grads = g.zeros_like()
        dpose = torch.zeros(V, 6, dtype=torch.float32, device=self.torch_device)
        gst = g.struct()
        gg = grads.grad_struct()
        c = lambda t: None if t is None else t.contiguous()
        dC, dD, dA = c(dC), c(dD), c(dA)
        npix = sum(cm.npix for cm in cams)
        _check_gaussians(g, self.torch_device)
        _need(poses.contiguous(), 16 * V, "poses", device=self.torch_device)
        _need(dC, 3 * npix, "dL_dcolor", device=self.torch_device)
        _need(dD, npix, "dL_ddepth", device=self.torch_device)
        _need(dA, npix, "dL_dalpha", device=self.torch_device)
        if state.numel() < self.state_bytes(cams, g.n, plan.pair_capacity, (plan.bin_w, plan.bin_h)):
            raise ValueError("state is smaller than the plan requires")
        rc = self.lib.gs_render_backward(self.h, ctypes.byref(gst), cam_array(cams), _p(poses.contiguous()), V,
                                         _p(state), state.numel(), ctypes.byref(plan), _p(dC), _p(dD), _p(dA),
                                         ctypes.byref(gg), _p(dpose), _stream())
        self._check(rc)
        return grads, dpose

    def reproj(self, cams, poses, points, uv, view_idx, delta: float, weight: float = 1.0,
               dpose: Optional[torch.Tensor] = None, point_grads: bool = False, noalloc: bool = False):
        """Returns (residual [M,2], loss [V], dpose [V,6]) (dpose accumulated),
        plus dL/dpoints [M,3] when ``point_grads``.  ``noalloc`` calls
        gs_reproj_residual_noalloc (the library's static scratch instead of
        the context's buffer; same results)."""
        cams = as_cameras(cams)
        V = len(cams)
        dev = self.torch_device
        points = points.contiguous()
        uv = uv.contiguous()
        view_idx = view_idx.to(torch.int32).contiguous()
        M = int(points.shape[0])
        _need(poses.contiguous(), 16 * V, "poses", device=dev)
        _need(points, 3 * M, "points", device=dev)
        _need(uv, 2 * M, "uv", device=dev)
        _need(view_idx, M, "view_idx", dtype=torch.int32, device=dev)
        _need(dpose, 6 * V, "dpose", device=dev)
        residual = torch.empty(max(M, 1), 2, dtype=torch.float32, device=dev)
        loss = torch.empty(V, dtype=torch.float32, device=dev)
        if dpose is None:
            dpose = torch.zeros(V, 6, dtype=torch.float32, device=dev)
        dpts = torch.empty(max(M, 1), 3, dtype=torch.float32, device=dev) if point_grads else None
        fn = self.lib.gs_reproj_residual_noalloc if noalloc else self.lib.gs_reproj_residual
        rc = fn(self.h, cam_array(cams), _p(poses.contiguous()), V, _p(points), _p(uv), _p(view_idx), M,
                float(delta), float(weight), _p(residual), _p(loss), _p(dpose), _p(dpts), _stream())
        self._check(rc)
        if point_grads:
            return residual[:M], loss, dpose, dpts[:M]
        return residual[:M], loss, dpose

    def pose_retract(self, poses: torch.Tensor, xi: torch.Tensor) -> torch.Tensor:
        """Exp(xi[v]) poses[v] per view (see gs_pose_retract): poses [V,16] or
        [V,4,4], xi [V,6]; returns a new [V,16] tensor."""
        dev = self.torch_device
        poses = poses.reshape(-1, 16).contiguous()
        V = int(poses.shape[0])
        xi = xi.detach().to(torch.float32).contiguous()
        _need(poses, 16 * V, "poses", device=dev)
        _need(xi, 6 * V, "xi", device=dev)
        out = torch.empty_like(poses)
        self._check(self.lib.gs_pose_retract(self.h, V, _p(poses), _p(xi), _p(out), _stream()))
        return out

    def pose_tangent_grad(self, xi: torch.Tensor, dpose: torch.Tensor) -> torch.Tensor:
        """J_l(xi)^T dpose per view (see gs_pose_tangent_grad)."""
        dev = self.torch_device
        xi = xi.detach().to(torch.float32).contiguous()
        dpose = dpose.to(torch.float32).contiguous()
        V = int(xi.numel() // 6)
        _need(xi, 6 * V, "xi", device=dev)
        _need(dpose, 6 * V, "dpose", device=dev)
        out = torch.empty(V, 6, dtype=torch.float32, device=dev)
        self._check(self.lib.gs_pose_tangent_grad(self.h, V, _p(xi), _p(dpose), _p(out), _stream()))
        return out

    def adam_update(self, g: "Gaussians", grads: Optional["Gaussians"], adam, opts: "StepOptions",
                    poses: Optional[torch.Tensor] = None, dpose: Optional[torch.Tensor] = None):
        """The optimiser of gs_mapping_step on caller-given gradients (see
        gs_adam_update): ``adam`` = (m, v, step) laid out for g.n Gaussians
        and V poses, step an int32[2] (Gaussian, pose updates); updates g's
        tensors and ``poses`` ([V,16]) in place."""
        dev = self.torch_device
        _check_gaussians(g, dev)
        m, v, step = adam
        V = 0 if poses is None else int(poses.numel() // 16)
        na = g.n * g.floats_per_gaussian + 6 * V
        _need(m, na, "adam m", device=dev)
        _need(v, na, "adam v", device=dev)
        _need(step, 2, "adam step", dtype=torch.int32, device=dev)
        if opts.update_gaussians:
            if grads is None:
                raise ValueError("update_gaussians needs the gradients")
            _check_gaussians(grads, dev)
        if opts.update_poses and V:
            if dpose is None or not poses.is_contiguous():
                raise ValueError("update_poses needs contiguous poses and dpose")
            _need(dpose.contiguous(), 6 * V, "dpose", device=dev)
        gst = g.struct()
        gg = grads.grad_struct() if grads is not None else None
        ad = A.gs_adam(_p(m), _p(v), _p(step))
        o = opts.struct(0, (0, 0))
        rc = self.lib.gs_adam_update(self.h, ctypes.byref(gst), ctypes.byref(gg) if gg is not None else None,
                                     ctypes.byref(ad), _p(poses), _p(None if dpose is None else dpose.contiguous()),
                                     V, ctypes.byref(o), _stream())
        self._check(rc)

    def ssim(self, cams, img: torch.Tensor, ref: torch.Tensor, weights: Optional[torch.Tensor] = None,
             dimg: Optional[torch.Tensor] = None):
        """Mean SSIM per view of planar colour images (concatenated [3,H,W]
        per view) and, with ``weights`` ([V]), the gradient of
        sum_v weights[v] (1 - SSIM_v) accumulated into ``dimg`` (allocated
        zero if None).  Returns (ssim [V], dimg or None)."""
        cams = as_cameras(cams)
        V = len(cams)
        dev = self.torch_device
        npx = sum(c.npix for c in cams)
        img = img.contiguous()
        ref = ref.contiguous()
        _need(img, 3 * npx, "img", device=dev)
        _need(ref, 3 * npx, "ref", device=dev)
        ca = cam_array(cams)
        nbytes = int(self.lib.gs_ssim_workspace_bytes(ca, V))
        if nbytes == 0:
            raise GSError(A.GS_EINVAL, "bad cameras")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        out = torch.empty(V, dtype=torch.float32, device=dev)
        if weights is not None:
            weights = weights.to(torch.float32).contiguous()
            _need(weights, V, "weights", device=dev)
            if dimg is None:
                dimg = torch.zeros(3 * npx, dtype=torch.float32, device=dev)
            _need(dimg, 3 * npx, "dimg", device=dev)
        rc = self.lib.gs_ssim(self.h, ca, V, _p(img), _p(ref), _p(weights), _p(out), _p(dimg), _p(ws), nbytes,
                              _stream())
        self._check(rc)
        return out, dimg

    def prune(self, g: Gaussians, tau: float, adam: Optional[Tuple[torch.Tensor, torch.Tensor, torch.Tensor]] = None,
              V: int = 0):
        """Removes Gaussians with opacity below tau (see gs_prune).  ``adam``:
        optional (m, v, step) moments laid out for g.n Gaussians and V poses.
        Returns (pruned Gaussians, re-laid-out (m, v, step) or None); reads the
        kept count back (one synchronisation)."""
        dev = self.torch_device
        _check_gaussians(g, dev)
        out = g.like(*(torch.empty_like(t) for t in g.tensors()))
        nbytes = int(self.lib.gs_prune_workspace_bytes(g.n))
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
        nout = torch.zeros(1, dtype=torch.int64, device=dev)
        ain = aout = None
        if adam is not None:
            m, v, step = adam
            m2, v2 = torch.empty_like(m), torch.empty_like(v)
            ain = A.gs_adam(_p(m), _p(v), _p(step))
            aout = A.gs_adam(_p(m2), _p(v2), _p(step))
        gi, go = g.struct(), out.struct()
        rc = self.lib.gs_prune(self.h, ctypes.byref(gi), float(tau), ctypes.byref(go),
                               ctypes.byref(ain) if ain is not None else None,
                               ctypes.byref(aout) if aout is not None else None, int(V), _p(nout), _p(ws), nbytes,
                               _stream())
        self._check(rc)
        k = int(nout.item())
        pruned = g.like(*(t[:k] for t in out.tensors()))
        if adam is None:
            return pruned, None
        keep = k * g.floats_per_gaussian + 6 * V
        return pruned, (m2[:keep], v2[:keep], adam[2])

    def densify(self, g: Gaussians, capacity: int, cams, poses: torch.Tensor, alpha: torch.Tensor,
                tgt_color: torch.Tensor, tgt_depth: torch.Tensor, gamma: float = 0.99, all_pixels: bool = False,
                adam: Optional[Tuple[torch.Tensor, torch.Tensor, torch.Tensor]] = None):
        """Appends new Gaussians at under-reconstructed pixels (see
        gs_densify).  Allocates arrays for ``capacity`` Gaussians, copies g
        into them and appends in place.  Returns (Gaussians, (held, asked),
        grown (m, v, step) or None); one synchronisation for the counts."""
        cams = as_cameras(cams)
        V = len(cams)
        dev = self.torch_device
        _check_gaussians(g, dev)
        if capacity < g.n:
            raise ValueError("capacity below the current count")
        K = sh_coeffs(g.sh_degree)
        cap = g.like(torch.empty(capacity, 3, device=dev),
                     torch.empty(capacity, 1 if g.isotropic else 3, device=dev),
                     torch.empty(capacity, 0 if g.isotropic else 4, device=dev), torch.empty(capacity, device=dev),
                     torch.empty((capacity, 3) if g.sh_degree < 0 else (capacity, K, 3), device=dev))
        for dst, src in zip(cap.tensors(), g.tensors()):
            dst[:g.n].copy_(src.reshape(dst[:g.n].shape))
        gst = cap.struct()
        gst.n = g.n
        ca = cam_array(cams)
        nbytes = int(self.lib.gs_densify_workspace_bytes(ca, V))
        if nbytes == 0:
            raise GSError(A.GS_EINVAL, "bad cameras")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        counts = torch.zeros(2, dtype=torch.int64, device=dev)
        ain = aout = None
        if adam is not None:
            m, v, step = adam
            m2 = torch.empty(capacity * g.floats_per_gaussian + 6 * V, dtype=torch.float32, device=dev)
            v2 = torch.empty_like(m2)
            ain = A.gs_adam(_p(m), _p(v), _p(step))
            aout = A.gs_adam(_p(m2), _p(v2), _p(step))
        npx = sum(c.npix for c in cams)
        _need(alpha.contiguous(), npx, "alpha", device=dev)
        _need(tgt_color.contiguous(), 3 * npx, "tgt_color", device=dev)
        _need(tgt_depth.contiguous(), npx, "tgt_depth", device=dev)
        rc = self.lib.gs_densify(self.h, ca, _p(poses.contiguous()), V, _p(alpha.contiguous()),
                                 _p(tgt_color.contiguous()), _p(tgt_depth.contiguous()), float(gamma),
                                 int(all_pixels), ctypes.byref(gst), int(capacity),
                                 ctypes.byref(ain) if ain is not None else None,
                                 ctypes.byref(aout) if aout is not None else None, _p(counts), _p(ws), nbytes,
                                 _stream())
        self._check(rc)
        c0, c1 = (int(x) for x in counts.cpu())
        out = g.like(*(t[:c0] for t in cap.tensors()))
        if adam is None:
            return out, (c0, c1), None
        keep = c0 * g.floats_per_gaussian + 6 * V
        return out, (c0, c1), (m2[:keep], v2[:keep], adam[2])

    def _bin(self, bin):
        """Resolve (0, 0) to the context's bin choice (kept in Python too, so
        the state can be sized before the call)."""
        if tuple(bin) != (0, 0):
            return int(bin[0]), int(bin[1])
        return self.bin_choice

    def bin_records(self, cams, n: int, tile: Tuple[int, int], rect: torch.Tensor, depth: torch.Tensor,
                    capacity: int):
        """Binning stage alone for bins of ``tile`` = (w, h) pixels: returns
        (values [P] int64, ranges [bins,2] int64)."""
        cams = as_cameras(cams)
        V = len(cams)
        dev = self.torch_device
        nbytes = self.state_bytes(cams, n, capacity, tile)
        state = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        values = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
        ntiles = sum(-(-c.width // tile[0]) * -(-c.height // tile[1]) for c in cams)
        ranges = torch.empty(ntiles, 2, dtype=torch.int32, device=dev)
        npairs = ctypes.c_int64()
        rect = rect.contiguous()
        depth = depth.contiguous()
        _need(rect, 2 * V * n, "rect", dtype=rect.dtype, device=dev)
        if rect.dtype not in (torch.int32,):
            raise ValueError("rect must be int32 (bit pattern of the packed u32 rect)")
        _need(depth, V * n, "depth", device=dev)
        rc = self.lib.gs_bin_records(self.h, cam_array(cams), V, n, tile[0], tile[1], _p(rect), _p(depth),
                                     _p(values), capacity, _p(ranges), ctypes.byref(npairs), _p(state), nbytes,
                                     _stream())
        self._check(rc)
        P = int(npairs.value)
        u = lambda t: t.to(torch.int64) & 0xFFFFFFFF
        return u(values[:P]), u(ranges)

    def autotune(self, g: Gaussians, cams, poses, iters: int = 3):
        """Returns ((tile_w, tile_h), (bin_w, bin_h)) and makes them, and the
        backward tile (``bwd_tile_choice``), the context's choice."""
        cams = as_cameras(cams)
        tw, th, bw, bh = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        btw, bth = ctypes.c_int32(), ctypes.c_int32()
        gst = g.struct()
        _check_gaussians(g, self.torch_device)
        _need(poses.contiguous(), 16 * len(cams), "poses", device=self.torch_device)
        rc = self.lib.gs_autotune(self.h, ctypes.byref(gst), cam_array(cams), _p(poses.contiguous()), len(cams),
                                  iters, ctypes.byref(tw), ctypes.byref(th), ctypes.byref(bw), ctypes.byref(bh),
                                  ctypes.byref(btw), ctypes.byref(bth), _stream())
        self._check(rc)
        self.bin_choice = (int(bw.value), int(bh.value))
        self.bwd_tile_choice = (int(btw.value), int(bth.value))
        return (int(tw.value), int(th.value)), self.bin_choice


_default: Dict[int, Context] = {}


def default_context(device: Optional[int] = None) -> Context:
    d = torch.cuda.current_device() if device is None else int(device)
    if d not in _default:
        _default[d] = Context(d)
    return _default[d]


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------

class GSRenderFn(torch.autograd.Function):
    """Differentiable batched render: (means, log_scales, quats, opacity
    logits, colours, pose tangent xi [V,6], poses [V,16]) -> (colour, depth,
    alpha), concatenated over views.  The views are rendered at
    Exp(xi[v]) poses[v] (gs_pose_retract); the gradient with respect to xi is
    J_l(xi)^T times the left-perturbation gradient at the rendered pose
    (gs_pose_tangent_grad), so it is exact at any xi, and the plain
    left-perturbation gradient at xi = 0.  Inputs are saved with
    save_for_backward, so an in-place change between forward and backward
    raises."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, colors, pose_tangent, poses, gs_ctx, cams,
                sh_degree, isotropic, tile, sync):
        g = Gaussians(means.contiguous(), log_scales.contiguous(), quats.contiguous(), opacity_logits.contiguous(),
                      colors.contiguous(), sh_degree, isotropic)
        rposes = gs_ctx.pose_retract(poses, pose_tangent)
        color, depth, alpha, state, plan = gs_ctx.forward(g, cams, rposes, tile=tile, sync=sync)
        if not sync:
            gs_ctx.last_async_state = state
        ctx.save_for_backward(means, log_scales, quats, opacity_logits, colors, pose_tangent, rposes, state)
        ctx.gs = (gs_ctx, cams, sh_degree, isotropic, plan)
        return color, depth, alpha

    @staticmethod
    def backward(ctx, dC, dD, dA):
        means, log_scales, quats, opacity_logits, colors, pose_tangent, rposes, state = ctx.saved_tensors
        gs_ctx, cams, sh_degree, isotropic, plan = ctx.gs
        g = Gaussians(means.contiguous(), log_scales.contiguous(), quats.contiguous(), opacity_logits.contiguous(),
                      colors.contiguous(), sh_degree, isotropic)
        grads, dpose = gs_ctx.backward(g, cams, rposes, state, plan, dC, dD, dA)
        dxi = gs_ctx.pose_tangent_grad(pose_tangent, dpose)
        return (grads.means.view_as(means), grads.log_scales.view_as(log_scales), grads.quats.view_as(quats),
                grads.opacity_logits.view_as(opacity_logits), grads.colors.view_as(colors),
                dxi.view_as(pose_tangent), None, None, None, None, None, None, None)


def render(g: Gaussians, cams, poses: torch.Tensor, pose_tangent: Optional[torch.Tensor] = None,
           ctx: Optional[Context] = None, tile=(0, 0), sync: bool = True):
    """Differentiable render of V views at Exp(pose_tangent[v]) poses[v].
    Gradients flow to g's tensors (if they require grad) and to
    ``pose_tangent`` ([V,6], xi = (v, w), translation first; a zero tensor
    with requires_grad gives the left-perturbation gradient d/dxi at 0).
    sync=False renders without a host synchronisation, with the pair
    capacity the context estimated from earlier synchronous renders: a pair
    overflow then gives an empty render and zero gradients, flagged in the
    state that ``ctx.check_async()`` reads."""
    cams = as_cameras(cams)
    ctx = ctx or default_context()
    if pose_tangent is None:
        pose_tangent = torch.zeros(len(cams), 6, dtype=torch.float32, device=poses.device)
    return GSRenderFn.apply(g.means, g.log_scales, g.quats, g.opacity_logits, g.colors, pose_tangent,
                            poses.detach().reshape(len(cams), 16).contiguous(), ctx, cams, g.sh_degree, g.isotropic,
                            tuple(tile), bool(sync))


class SSIMLossFn(torch.autograd.Function):
    """Per-view SSIM loss 1 - SSIM_v of a planar colour render against a
    fixed reference (mapping loss, Sec. 3.4); differentiable in the render."""

    @staticmethod
    def forward(ctx, img, ref, gs_ctx, cams):
        s, _ = gs_ctx.ssim(cams, img.detach(), ref)
        ctx.save_for_backward(img, ref)
        ctx.gs_ctx, ctx.cams = gs_ctx, cams
        return 1.0 - s

    @staticmethod
    def backward(ctx, go):
        img, ref = ctx.saved_tensors
        _, d = ctx.gs_ctx.ssim(ctx.cams, img.detach(), ref, weights=go.contiguous())
        return d, None, None, None


def ssim_loss(img: torch.Tensor, ref: torch.Tensor, cams, ctx: Optional[Context] = None) -> torch.Tensor:
    """[V] tensor of 1 - SSIM per view (see gs_ssim for the definition)."""
    cams = as_cameras(cams)
    return SSIMLossFn.apply(img, ref.detach(), ctx or default_context(), cams)


# ---------------------------------------------------------------------------
# mapping / pose-refinement step
# ---------------------------------------------------------------------------

@dataclass
class StepOptions:
    w_color: float = 1.0
    w_depth: float = 0.1
    w_reproj: float = 0.0
    huber_delta: float = 2.0
    use_gate: bool = False
    gate_gamma: float = 0.99
    update_gaussians: bool = False
    update_poses: bool = False
    accumulate_grads: bool = False
    use_graph: bool = True
    lr_means: float = 1e-4
    lr_log_scales: float = 1e-3
    lr_quats: float = 1e-3
    lr_opacity: float = 5e-2
    lr_colors: float = 2.5e-3
    lr_pose: float = 1e-3
    adam_b1: float = 0.9
    adam_b2: float = 0.999
    adam_eps: float = 1e-8
    tile: Tuple[int, int] = (0, 0)
    bin: Tuple[int, int] = (0, 0)
    w_ssim: float = 0.0
    bwd_tile: Tuple[int, int] = (0, 0)

    def struct(self, capacity: int, bin=None) -> A.gs_step_opts:
        b = self.bin if bin is None else bin
        return A.gs_step_opts(self.w_color, self.w_depth, self.w_reproj, self.huber_delta, int(self.use_gate),
                              self.gate_gamma, int(self.update_gaussians), int(self.update_poses),
                              int(self.accumulate_grads), int(self.use_graph), self.lr_means, self.lr_log_scales,
                              self.lr_quats, self.lr_opacity, self.lr_colors, self.lr_pose, self.adam_b1,
                              self.adam_b2, self.adam_eps, self.tile[0], self.tile[1], b[0], b[1], capacity,
                              self.w_ssim, self.bwd_tile[0], self.bwd_tile[1])


# the paper's Fusion Bridge weights (Supplementary, hyper-parameter table):
# re-projection w1 = 1.5, colour w2 = 0.5, depth w3 = 1, border gate gamma = 0.99
PAPER_FUSION_BRIDGE = dict(w_reproj=1.5, w_color=0.5, w_depth=1.0, use_gate=True, gate_gamma=0.99)

# the paper's mapping loss (Sec. 3.4; hyper-parameter table): zeta = 0.3, depth
# w4 = 0.5, colour w5 = 1:  (1 - zeta)(w4 L1_D + w5 L1_C) + zeta L_SSIM, the pose
# held fixed
PAPER_MAPPING = dict(w_color=(1 - 0.3) * 1.0, w_depth=(1 - 0.3) * 0.5, w_reproj=0.0, w_ssim=0.3,
                     update_gaussians=True, update_poses=False)


class MappingStep:
    """Owns the device buffers of ``gs_mapping_step`` for one scene shape and
    enqueues one step per call (graph-captured by default)."""

    def __init__(self, ctx: Context, g: Gaussians, cams, poses: torch.Tensor, target_color: torch.Tensor,
                 target_depth: torch.Tensor, opts: StepOptions, mask: Optional[torch.Tensor] = None,
                 matches: Optional[Tuple[torch.Tensor, torch.Tensor, torch.Tensor]] = None,
                 capacity: Optional[int] = None):
        self.ctx = ctx
        self.g = g
        self.cams = as_cameras(cams)
        self.V = len(self.cams)
        self.opts = opts
        dev = ctx.torch_device
        self.poses = poses.reshape(self.V, 16).contiguous()
        self.tc = target_color.contiguous()
        self.td = target_depth.contiguous()
        self.mask = None if mask is None else mask.contiguous()
        if matches is not None:
            self.points, self.uv, self.vidx = (matches[0].contiguous(), matches[1].contiguous(),
                                               matches[2].to(torch.int32).contiguous())
            self.M = int(self.points.shape[0])
        else:
            self.points = self.uv = self.vidx = None
            self.M = 0
        npix_ = sum(c.npix for c in self.cams)
        _check_gaussians(g, dev)
        _need(self.poses, 16 * self.V, "poses", device=dev)
        _need(self.tc, 3 * npix_, "target_color", device=dev)
        _need(self.td, npix_, "target_depth", device=dev)
        _need(self.mask, npix_, "mask", device=dev)
        if self.M:
            _need(self.points, 3 * self.M, "points", device=dev)
            _need(self.uv, 2 * self.M, "uv", device=dev)
            _need(self.vidx, self.M, "view_idx", dtype=torch.int32, device=dev)
        self.bin = ctx._bin(opts.bin)
        if capacity is None:
            # size from one counting forward pass
            _, _, _, _, plan = ctx.forward(g, self.cams, self.poses, tile=opts.tile, bin=self.bin)
            capacity = int(plan.n_pairs * 1.3) + 4096
        self.capacity = int(capacity)
        npix = sum(c.npix for c in self.cams)
        self.ws_bytes = ctx.workspace_bytes(self.cams, g.n, g.sh_degree, self.capacity, self.bin)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.ws[:64].zero_()     # the status words (the sticky flags start at zero)
        self.grads = g.zeros_like()
        na = g.n * g.floats_per_gaussian + 6 * self.V
        self.adam_m = torch.zeros(na, dtype=torch.float32, device=dev)
        self.adam_v = torch.zeros(na, dtype=torch.float32, device=dev)
        self.adam_step = torch.zeros(2, dtype=torch.int32, device=dev)   # Gaussian updates, pose updates
        self.color = torch.empty(3 * npix, dtype=torch.float32, device=dev)
        self.depth = torch.empty(npix, dtype=torch.float32, device=dev)
        self.alpha = torch.empty(npix, dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1 + 4 * self.V, dtype=torch.float32, device=dev)
        self.dpose = torch.zeros(self.V, 6, dtype=torch.float32, device=dev)
        self._build_structs()

    def _build_structs(self):
        self._gst = self.g.struct()
        self._gg = self.grads.grad_struct()
        self._adam = A.gs_adam(_p(self.adam_m), _p(self.adam_v), _p(self.adam_step))
        self._ca = cam_array(self.cams)
        self._tg = A.gs_targets(_p(self.tc), _p(self.td), _p(self.mask))
        self._mt = A.gs_matches(_p(self.points), _p(self.uv), _p(self.vidx), self.M)
        self._opts = self.opts.struct(self.capacity, self.bin)

    def set_options(self, opts: StepOptions):
        if self.ctx._bin(opts.bin) != self.bin:
            raise ValueError("the bin size is fixed when the workspace is sized")
        self.opts = opts
        self._opts = opts.struct(self.capacity, self.bin)

    def __call__(self):
        rc = self.ctx.lib.gs_mapping_step(self.ctx.h, ctypes.byref(self._gst), ctypes.byref(self._gg),
                                          ctypes.byref(self._adam), self._ca, _p(self.poses), self.V,
                                          ctypes.byref(self._tg), ctypes.byref(self._mt), ctypes.byref(self._opts),
                                          _p(self.ws), self.ws_bytes, _p(self.color), _p(self.depth),
                                          _p(self.alpha), _p(self.loss), _p(self.dpose), _stream())
        self.ctx._check(rc)

    def profile(self, counts: bool = True):
        """One eager step with per-stage HIP-event timing on the current
        stream.  Returns ({stage: ms}, (visited, blended) or None)."""
        L = self.ctx.lib
        ns = L.gs_num_stages()
        ms = (ctypes.c_float * ns)()
        fc = (ctypes.c_int64 * 4)()
        o = self.opts.struct(self.capacity, self.bin)
        o.use_graph = 0
        rc = L.gs_step_profile(self.ctx.h, ctypes.byref(self._gst), ctypes.byref(self._gg), ctypes.byref(self._adam),
                               self._ca, _p(self.poses), self.V, ctypes.byref(self._tg), ctypes.byref(self._mt),
                               ctypes.byref(o), _p(self.ws), self.ws_bytes, _p(self.color), _p(self.depth),
                               _p(self.alpha), _p(self.loss), _p(self.dpose), ms, fc if counts else None, _stream())
        self.ctx._check(rc)
        names = [L.gs_stage_name(i).decode() for i in range(ns)]
        return dict(zip(names, list(ms))), (tuple(int(x) for x in fc) if counts else None)

    def status(self) -> Dict[str, int]:
        """Flags of every step since the previous call (bit 0 pair overflow,
        bit 1 binning scan timed out, bit 2 non-finite parameter; a flagged
        step made no update), and the last step's pair and visible counts.
        Synchronises the stream and clears the sticky flags."""
        fl = ctypes.c_int32()
        npairs = ctypes.c_int64()
        nvis = ctypes.c_int64()
        rc = self.ctx.lib.gs_step_status(self.ctx.h, _p(self.ws), self.ws_bytes, ctypes.byref(fl),
                                         ctypes.byref(npairs), ctypes.byref(nvis), _stream())
        self.ctx._check(rc)
        return {"flags": int(fl.value), "n_pairs": int(npairs.value), "n_visible": int(nvis.value)}

    def check(self) -> Dict[str, int]:
        """status(), raising GSError when a step since the previous check was
        flagged."""
        st = self.status()
        f = st["flags"]
        if f & 1:
            raise GSError(A.GS_ECAPACITY, f"{st['n_pairs']} pairs exceed the capacity {self.capacity}; "
                                          "re-plan the step with a larger capacity")
        if f & 4:
            raise GSError(A.GS_EINVAL, "a Gaussian parameter is not finite; the flagged steps made no update")
        if f:
            raise GSError(A.GS_EDEVICE, f"step status flags {f:#x}")
        return st


class JointRefinement:
    """The alternating optimisation of the paper on one ``MappingStep``: k_pose
    pose-refinement iterations with the Fusion Bridge loss (re-projection +
    rendering terms, filter gate; Sec. 3.3, Gaussians held fixed), then k_map
    mapping iterations with the mapping loss (Sec. 3.4, poses held fixed).
    Both phases share the step's buffers and Adam state (pose and Gaussian
    moments live in separate slots; the bias-correction counter is shared);
    each phase's step is captured as its own hipGraph."""

    def __init__(self, step: "MappingStep", pose_opts: Optional[StepOptions] = None,
                 map_opts: Optional[StepOptions] = None):
        from dataclasses import replace
        base = step.opts
        self.step = step
        self.pose_opts = pose_opts or replace(base, **PAPER_FUSION_BRIDGE, w_ssim=0.0, update_poses=True,
                                              update_gaussians=False)
        self.map_opts = map_opts or replace(base, **PAPER_MAPPING)

    def __call__(self, k_pose: int, k_map: int):
        """Runs the two phases, then reads the step status once (one
        synchronisation) and raises GSError if any step was flagged (such
        steps made no update)."""
        self.step.set_options(self.pose_opts)
        for _ in range(k_pose):
            self.step()
        self.step.set_options(self.map_opts)
        for _ in range(k_map):
            self.step()
        self.step.check()


def select_viewpoints(covis, n_obs, alpha: float = 0.75, beta: int = 20):
    """Viewpoint selection of the Fusion Bridge (see gs_select_viewpoints):
    ``covis`` [F,F] feature matches between keyframes, ``n_obs`` [F] matched
    map points per keyframe.  Returns a bool array [F]."""
    import numpy as np
    covis = np.ascontiguousarray(covis, dtype=np.int32)
    n_obs = np.ascontiguousarray(n_obs, dtype=np.int32)
    F = int(n_obs.shape[0])
    if covis.shape != (F, F):
        raise ValueError("covis must be [F, F]")
    out = np.zeros(F, np.int32)
    rc = A.load().gs_select_viewpoints(covis.ctypes.data, n_obs.ctypes.data, F, float(alpha), int(beta),
                                       out.ctypes.data)
    if rc != 0:
        raise GSError(rc, "gs_select_viewpoints rejected its arguments")
    return out.astype(bool)

