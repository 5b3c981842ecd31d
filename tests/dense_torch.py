"""Dense, tile-free renderer in torch (CPU, FP64), differentiated by autograd.

Used only to pin the oracle: every Gaussian is evaluated at every pixel (no
support rect, no buckets), rotations come from ``torch.linalg.matrix_exp`` of
the quaternion's axis-angle, the EWA Jacobian from ``torch.func.jacrev`` of
the pinhole projection, the SH basis from associated Legendre polynomials,
the pose perturbation from ``matrix_exp`` of the twist, and every gradient
from autograd.  Front-to-back blending follows the colour / depth / border
mask compositing equations of Sec. 3.3-3.4 with the clamp 0.99, the 1/255
skip and the 1e-4 termination; the discrete decisions are held constant.
The EWA Jacobian is taken at the camera-space point whose x/z and y/z are
clamped at 1.3 times the half field of view (the projected mean itself is
not clamped), so autograd sees no derivative through a clamped coordinate.
"""
import math

import numpy as np
import torch

ZNEAR = 0.2
JCLAMP = 1.3


def _hat(w):
    z = torch.zeros((), dtype=w.dtype)
    return torch.stack([torch.stack([z, -w[2], w[1]]), torch.stack([w[2], z, -w[0]]),
                        torch.stack([-w[1], w[0], z])])


def twist_exp(xi):
    M = torch.zeros((4, 4), dtype=xi.dtype)
    M = M.clone()
    top = torch.cat([_hat(xi[3:]), xi[:3].reshape(3, 1)], dim=1)
    M = torch.cat([top, torch.zeros((1, 4), dtype=xi.dtype)], dim=0)
    return torch.linalg.matrix_exp(M)


def quat_to_R(q):
    """Rotation of the unit quaternion q/|q| = (cos(a/2), sin(a/2) n) as exp(a [n]x)."""
    qh = q / torch.linalg.norm(q)
    vn = torch.linalg.norm(qh[1:])
    ang = 2.0 * torch.atan2(vn, qh[0])
    axis = qh[1:] / vn
    return torch.linalg.matrix_exp(_hat(axis * ang))


def _legendre(l, m, x):
    s = torch.sqrt(1 - x * x)
    table = {
        (0, 0): lambda: torch.ones_like(x),
        (1, 0): lambda: x, (1, 1): lambda: -s,
        (2, 0): lambda: 0.5 * (3 * x * x - 1), (2, 1): lambda: -3 * x * s, (2, 2): lambda: 3 * (1 - x * x),
        (3, 0): lambda: 0.5 * (5 * x ** 3 - 3 * x), (3, 1): lambda: -1.5 * (5 * x * x - 1) * s,
        (3, 2): lambda: 15 * x * (1 - x * x), (3, 3): lambda: -15 * s ** 3,
    }
    return table[(l, m)]()


def real_sh(deg, d, signs=None):
    """Real orthonormal SH of unit directions d [..,3] from associated
    Legendre polynomials; index l*l + l + m.  ``signs`` (per index) picks the
    sign convention."""
    ct = d[..., 2]
    phi = torch.atan2(d[..., 1], d[..., 0])
    out = []
    for l in range(deg + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            N = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            P = _legendre(l, am, ct)
            if m == 0:
                y = N * P
            elif m > 0:
                y = math.sqrt(2) * N * P * torch.cos(m * phi)
            else:
                y = math.sqrt(2) * N * P * torch.sin(am * phi)
            out.append(y)
    Y = torch.stack(out, dim=-1)
    if signs is not None:
        Y = Y * torch.as_tensor(signs, dtype=Y.dtype)
    return Y


def render_dense(means, log_scales, quats, opl, colors, sh_degree, cam, T_cw, xi=None, sh_signs=None,
                 stats=None):
    """Returns (C [3,H,W], D [H,W], A [H,W]) as differentiable torch tensors.
    All inputs are torch float64 tensors; ``xi`` (6,) perturbs the pose as
    Exp(xi) T_cw.  ``stats`` (a dict, optional) receives how often the
    discrete branches were taken: 'alpha_clamped' fragments blended with
    o exp(-sigma) > 0.99, 'terminated' pixels that stopped before a candidate
    with alpha >= 1/255, 'jclamped' Gaussians whose Jacobian point was
    clamped, 'jclamped_blended' fragments of those."""
    W, H = cam.width, cam.height
    fx, fy, cx, cy = cam.fx, cam.fy, cam.cx, cam.cy
    T = T_cw if xi is None else twist_exp(xi) @ T_cw
    Rw, tw = T[:3, :3], T[:3, 3]
    n = means.shape[0]
    p = means @ Rw.T + tw
    assert bool((p[:, 2] > ZNEAR).all()), "dense renderer expects every Gaussian in front of the near plane"

    def proj(pt):
        return torch.stack([fx * pt[0] / pt[2] + cx, fy * pt[1] / pt[2] + cy])

    mu2 = torch.stack([proj(p[i]) for i in range(n)])
    # the Jacobian of the pinhole projection, taken where x/z and y/z are
    # clamped to the widened field of view
    limx = JCLAMP * W / (2.0 * fx)
    limy = JCLAMP * H / (2.0 * fy)
    xz = torch.clamp(p[:, 0] / p[:, 2], -limx, limx)
    yz = torch.clamp(p[:, 1] / p[:, 2], -limy, limy)
    pj = torch.stack([xz * p[:, 2], yz * p[:, 2], p[:, 2]], dim=1)
    J = torch.func.vmap(torch.func.jacrev(proj))(pj)   # [n,2,3]
    jcl = ((p[:, 0] / p[:, 2]).abs() > limx) | ((p[:, 1] / p[:, 2]).abs() > limy)
    Rs = torch.stack([quat_to_R(quats[i]) for i in range(n)])
    s2 = torch.exp(2 * log_scales)
    Sig = Rs @ torch.diag_embed(s2) @ Rs.transpose(1, 2)
    Sc = Rw @ Sig @ Rw.T
    S2 = J @ Sc @ J.transpose(1, 2) + 0.3 * torch.eye(2, dtype=means.dtype)
    Q = torch.linalg.inv(S2)
    o = torch.sigmoid(opl)
    if sh_degree < 0:
        col = colors
    else:
        Cc = -Rw.T @ tw
        dvec = means - Cc
        dn = dvec / torch.linalg.norm(dvec, dim=1, keepdim=True)
        Y = real_sh(sh_degree, dn, sh_signs)                      # [n,K]
        raw = torch.einsum("nk,nkc->nc", Y, colors) + 0.5
        col = torch.clamp(raw, min=0.0)
    z = p[:, 2]
    order = torch.argsort(z.detach(), stable=True)
    ys, xs = torch.meshgrid(torch.arange(H, dtype=means.dtype), torch.arange(W, dtype=means.dtype), indexing="ij")
    pix = torch.stack([xs.reshape(-1), ys.reshape(-1)], dim=1)   # [P,2]
    d = pix[:, None, :] - mu2[order][None, :, :]                 # [P,n,2]
    Qo = Q[order]
    sig = 0.5 * torch.einsum("pni,nij,pnj->pn", d, Qo, d)
    rawa = o[order][None, :] * torch.exp(-sig)
    alpha = torch.clamp(rawa, max=0.99)
    keep = ((alpha >= 1.0 / 255.0) & (sig >= 0)).detach()
    a = torch.where(keep, alpha, torch.zeros_like(alpha))
    one_m = 1 - a
    incl = torch.cumprod(one_m, dim=1)
    live = (incl >= 1e-4).detach()          # termination: T' < 1e-4 stops (T is non-increasing)
    a = torch.where(live, a, torch.zeros_like(a))
    one_m = 1 - a
    Tincl = torch.cumprod(one_m, dim=1)
    Texcl = torch.cat([torch.ones_like(Tincl[:, :1]), Tincl[:, :-1]], dim=1)
    w = a * Texcl
    C = w @ col[order]                       # [P,3]
    D = w @ z[order]
    A = 1 - Tincl[:, -1]
    if stats is not None:
        blended = (a > 0).detach()
        stats["alpha_clamped"] = int((blended & (rawa.detach() > 0.99)).sum())
        stats["terminated"] = int((keep & ~live).any(dim=1).sum())
        stats["jclamped"] = int(jcl.sum())
        stats["jclamped_blended"] = int((blended & jcl[order][None, :]).sum())
    return C.T.reshape(3, H, W), D.reshape(H, W), A.reshape(H, W)


def torch_params(g):
    """Leaf tensors (requires_grad) from an oracle.Gaussians."""
    t = lambda a: torch.tensor(np.asarray(a), dtype=torch.float64, requires_grad=True)
    return t(g.means), t(g.log_scales), t(g.quats), t(g.opacity_logits), t(g.colors)
