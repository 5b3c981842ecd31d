"""Pins of the FP64 oracle against what the paper and the mathematics fix.

No test here retypes an oracle formula to compare it with itself: each one
checks the oracle against a closed form of the paper's equations, an
invariant, a library routine, brute force, or finite differences.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

from synth import scenes
from tests import dense_torch as DT

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _one(oracle, mean, log_scale, quat=(1, 0, 0, 0), opl=2.0, col=(0.2, 0.5, 0.9)):
    return oracle.Gaussians(np.array([mean]), np.array([log_scale]), np.array([quat]), np.array([opl]),
                            np.array([col]))


def _cam(W=64, H=48, f=60.0, cx=32.0, cy=24.0):
    return scenes.Camera(W, H, f, f, cx, cy)


# --------------------------------------------------------------------------
# projection (Sec. 3.4 projection equation and its local-affine footprint)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("z,s", [(2.0, 0.05), (3.5, 0.02), (1.2, 0.1)])
def test_isotropic_on_axis_radius_matches_paper(oracle, z, s):
    """On the optical axis an isotropic Gaussian of radius r at depth d has a
    2D footprint r2D = f r / d (Sec. 3.4 projection equation); the EWA
    covariance is then (f r / d)^2 I, plus the 0.3 px^2 dilation."""
    cam = _cam()
    g = _one(oracle, (0.0, 0.0, z), (math.log(s),) * 3, quat=(0.3, -0.5, 0.7, 0.1))
    rec = oracle.project(g, cam, np.eye(4))[0]
    r2d = cam.fx * s / z
    assert rec[0] == 1
    assert rec[1] == pytest.approx(cam.cx) and rec[2] == pytest.approx(cam.cy)
    assert rec[16] - 0.3 == pytest.approx(r2d ** 2, rel=1e-12)
    assert rec[18] - 0.3 == pytest.approx(r2d ** 2, rel=1e-12)
    assert abs(rec[17]) < 1e-13 * r2d ** 2
    assert rec[10] == z


def test_densification_radius_is_one_pixel(oracle):
    """Sec. 3.4 densification: a new Gaussian gets the radius d / f, which by
    the projection equation is a 1 px footprint (1 + 0.3 after dilation)."""
    cam = _cam(f=525.0, W=640, H=480, cx=320, cy=240)
    for d in (0.7, 2.0, 4.5):
        g = _one(oracle, (0.0, 0.0, d), (math.log(d / cam.fx),) * 3)
        rec = oracle.project(g, cam, np.eye(4))[0]
        assert rec[16] == pytest.approx(1.0 + 0.3, rel=1e-12)


def test_projected_mean_shift_under_translation(oracle):
    """Moving the camera by delta along x shifts the projected mean of a point
    at depth z by f delta / z (pinhole projection of Sec. 3.2 / 3.4)."""
    cam = _cam()
    g = _one(oracle, (0.1, -0.2, 2.5), (math.log(0.05),) * 3)
    T = np.eye(4)
    T[0, 3] = 0.1
    r0 = oracle.project(g, cam, np.eye(4))[0]
    r1 = oracle.project(g, cam, T)[0]
    assert r1[1] - r0[1] == pytest.approx(cam.fx * 0.1 / 2.5, rel=1e-12)
    assert r1[2] == pytest.approx(r0[2], abs=1e-12)


def test_anisotropic_covariance_vs_scipy_rotation_and_fd_jacobian(oracle):
    """Sigma_2D = J R_cw R diag(s^2) R^T R_cw^T J^T + 0.3 I with R from
    scipy's quaternion convention and J the finite-difference Jacobian of the
    oracle's own projected mean w.r.t. the camera-space point."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(0)
    cam = _cam()
    for _ in range(20):
        mu = np.array([rng.uniform(-0.5, 0.5), rng.uniform(-0.4, 0.4), rng.uniform(1.5, 4)])
        ls = rng.normal(-3, 0.5, 3)
        q = rng.standard_normal(4)
        g = _one(oracle, mu, ls, quat=q)
        rec = oracle.project(g, cam, np.eye(4))[0]
        R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()   # scipy: scalar last
        Sig = R @ np.diag(np.exp(2 * ls)) @ R.T
        J = np.zeros((2, 3))
        h = 1e-6
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            rp = oracle.project(_one(oracle, mu + e, ls, quat=q), cam, np.eye(4))[0]
            rm = oracle.project(_one(oracle, mu - e, ls, quat=q), cam, np.eye(4))[0]
            J[:, k] = (rp[1:3] - rm[1:3]) / (2 * h)
        S2 = J @ Sig @ J.T
        got = np.array([[rec[16] - 0.3, rec[17]], [rec[17], rec[18] - 0.3]])
        np.testing.assert_allclose(got, S2, rtol=1e-7, atol=1e-9)
        # conic is the inverse of the dilated covariance
        Qm = np.linalg.inv(S2 + 0.3 * np.eye(2))
        np.testing.assert_allclose([rec[3], rec[4], rec[5]], [Qm[0, 0], Qm[0, 1], Qm[1, 1]], rtol=1e-6)


def test_isotropic_is_invariant_to_quaternion(oracle):
    cam = _cam()
    rng = np.random.default_rng(1)
    recs = [oracle.project(_one(oracle, (0.3, 0.1, 2.0), (-3.0,) * 3, quat=rng.standard_normal(4)), cam,
                           np.eye(4))[0] for _ in range(5)]
    for r in recs[1:]:
        np.testing.assert_allclose(r, recs[0], rtol=1e-12, atol=1e-14)


def test_near_plane_and_low_opacity_cull(oracle):
    cam = _cam()
    g = oracle.Gaussians(np.array([[0, 0, 0.2], [0, 0, 0.21], [0, 0, 2.0], [0, 0, 2.0]]),
                         np.full((4, 3), -3.0), np.tile([1.0, 0, 0, 0], (4, 1)),
                         np.array([2.0, 2.0, math.log((1 / 255 * 0.999) / (1 - 1 / 255 * 0.999)), 0.0]),
                         np.full((4, 3), 0.5))
    rec = oracle.project(g, cam, np.eye(4))
    assert list(rec[:, 0]) == [0, 1, 0, 1]


# --------------------------------------------------------------------------
# compositing (Sec. 3.4 colour and depth equations; Sec. 3.3 border mask)
# --------------------------------------------------------------------------

def test_single_isotropic_gaussian_closed_form(oracle):
    """One isotropic Gaussian on the axis: the paper's 2D kernel
    f(p) = o exp(-|p - mu2D|^2 / (2 r2D^2)) with r2D = f r / d (plus the
    dilation), clamped at 0.99 and cut below 1/255.  C = c f, D = d f,
    M_b = f."""
    cam = _cam()
    z, s, opl = 2.0, 0.05, 0.3
    col = np.array([0.2, 0.5, 0.9])
    g = _one(oracle, (0.0, 0.0, z), (math.log(s),) * 3, opl=opl, col=col)
    out = oracle.render(g, cam, np.eye(4))
    o = 1 / (1 + math.exp(-opl))
    var = (cam.fx * s / z) ** 2 + 0.3
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    f = o * np.exp(-((xs - cam.cx) ** 2 + (ys - cam.cy) ** 2) / (2 * var))
    f = np.minimum(f, 0.99)
    f[f < 1 / 255] = 0
    np.testing.assert_allclose(out["alpha"], f, atol=1e-14)
    np.testing.assert_allclose(out["depth"], z * f, atol=1e-13)
    for k in range(3):
        np.testing.assert_allclose(out["color"][k], col[k] * f, atol=1e-14)


def test_two_gaussians_blend(oracle):
    """C = c1 a1 + c2 a2 (1 - a1) for the nearer Gaussian 1 (colour equation)."""
    cam = _cam()
    c1, c2 = np.array([1.0, 0.0, 0.2]), np.array([0.0, 1.0, 0.4])
    g = oracle.Gaussians(np.array([[0.0, 0.0, 3.0], [0.0, 0.0, 2.0]]), np.full((2, 3), math.log(0.06)),
                         np.tile([1.0, 0, 0, 0], (2, 1)), np.array([0.5, -0.2]), np.stack([c2, c1]))
    out = oracle.render(g, cam, np.eye(4))
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]

    def a(z, opl):
        var = (cam.fx * 0.06 / z) ** 2 + 0.3
        v = np.minimum(1 / (1 + math.exp(-opl)) * np.exp(-((xs - 32) ** 2 + (ys - 24) ** 2) / (2 * var)), 0.99)
        v[v < 1 / 255] = 0
        return v

    a1, a2 = a(2.0, -0.2), a(3.0, 0.5)
    for k in range(3):
        np.testing.assert_allclose(out["color"][k], c1[k] * a1 + c2[k] * a2 * (1 - a1), atol=1e-14)
    np.testing.assert_allclose(out["depth"], 2.0 * a1 + 3.0 * a2 * (1 - a1), atol=1e-13)
    np.testing.assert_allclose(out["alpha"], 1 - (1 - a1) * (1 - a2), atol=1e-14)


def test_translated_camera_closed_form(oracle):
    """A camera translation of delta moves an isotropic Gaussian at depth z
    off the axis: its mean lands f delta / z pixels over (here 4 px) and its
    local-affine footprint becomes s^2 J J^T with the pinhole Jacobian
    J = [[f/z, 0, -f delta/z^2], [0, f/z, 0]] (closed form of EWA for an
    isotropic covariance)."""
    cam = _cam()
    z, s = 3.0, 0.05
    g = _one(oracle, (0.0, 0.0, z), (math.log(s),) * 3)
    T = np.eye(4)
    d = 4 * z / cam.fx
    T[0, 3] = d
    a1 = oracle.render(g, cam, T)["alpha"]
    f = cam.fx
    S = s * s * np.array([[f * f / z ** 2 + f * f * d * d / z ** 4, 0], [0, f * f / z ** 2]]) + 0.3 * np.eye(2)
    Qm = np.linalg.inv(S)
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    dx, dy = xs - (cam.cx + 4.0), ys - cam.cy
    o = 1 / (1 + math.exp(-2.0))
    a = np.minimum(o * np.exp(-0.5 * (Qm[0, 0] * dx * dx + Qm[1, 1] * dy * dy)), 0.99)
    a[a < 1 / 255] = 0
    np.testing.assert_allclose(a1, a, atol=1e-13)


def test_invariants_random_scene(oracle):
    """T non-increasing so alpha = 1 - T_final <= 1 - 1e-4; colour and depth
    are convex combinations scaled by alpha."""
    s = scenes.c1(n=400, seed=11)
    g = oracle.Gaussians.from_scene(s)
    out = oracle.render(g, s.cams[0], s.poses[0])
    A = out["alpha"]
    assert A.max() <= 1 - 1e-4 + 1e-15 and A.min() >= 0
    np.testing.assert_allclose(out["tfinal"], 1 - A, atol=1e-15)
    rec = oracle.project(g, s.cams[0], s.poses[0])
    vis = rec[:, 0] == 1
    cmin, cmax = g.colors[vis].min(0), g.colors[vis].max(0)
    for k in range(3):
        assert np.all(out["color"][k] <= cmax[k] * A + 1e-12)
        assert np.all(out["color"][k] >= cmin[k] * A - 1e-12)
    zs = rec[vis, 10]
    assert np.all(out["depth"] <= zs.max() * A + 1e-12) and np.all(out["depth"] >= zs.min() * A - 1e-12)


def test_pixel_list_equals_full_image(oracle):
    s = scenes.c1(n=300, width=70, height=45, seed=5)
    g = oracle.Gaussians.from_scene(s)
    full = oracle.render(g, s.cams[0], s.poses[0])
    pix = scenes.sample_pixels(s.cams[0], 200, 3)
    part = oracle.render(g, s.cams[0], s.poses[0], pixels=pix)
    np.testing.assert_array_equal(part["color"], full["color"][:, pix[:, 1], pix[:, 0]])
    np.testing.assert_array_equal(part["depth"], full["depth"][pix[:, 1], pix[:, 0]])


# --------------------------------------------------------------------------
# dense tile-free brute force in torch FP64 (forward and autograd gradients)
# --------------------------------------------------------------------------

def _tiny_scene(seed, n=48, W=32, H=24, sh_degree=-1):
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-0.6, 0.6, n), rng.uniform(-0.45, 0.45, n), rng.uniform(1.5, 4.0, n)], 1)
    ls = rng.normal(-2.6, 0.4, (n, 3))
    q = rng.standard_normal((n, 4))
    opl = rng.normal(0.5, 1.0, n)
    if sh_degree < 0:
        col = rng.uniform(0, 1, (n, 3))
    else:
        K = (sh_degree + 1) ** 2
        col = rng.normal(0, 0.2, (n, K, 3))
        col[:, 0] = rng.uniform(0, 1, (n, 3))
    cam = scenes.Camera(W, H, 30.0, 31.0, W / 2 - 0.3, H / 2 + 0.2)
    D = np.eye(4)
    from scipy.spatial.transform import Rotation
    D[:3, :3] = Rotation.from_rotvec(rng.normal(0, 0.05, 3)).as_matrix()
    D[:3, 3] = rng.normal(0, 0.05, 3)
    return means, ls, q, opl, col, cam, D


def _sh_signs(oracle, deg):
    """Sign convention of the oracle's basis relative to the Legendre one."""
    rng = np.random.default_rng(9)
    d = rng.standard_normal((64, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Yo = oracle.sh_basis(deg, d)
    Yt = DT.real_sh(deg, torch.tensor(d)).numpy()
    return np.sign(np.sum(Yo * Yt, axis=0))


@pytest.mark.parametrize("seed,sh", [(0, -1), (1, -1), (2, 3), (3, 1)])
def test_dense_brute_force_forward_and_autograd(oracle, seed, sh):
    means, ls, q, opl, col, cam, T = _tiny_scene(seed, sh_degree=sh)
    g = oracle.Gaussians(means, ls, q, opl, col, sh)
    out = oracle.render(g, cam, T)
    signs = _sh_signs(oracle, sh) if sh >= 0 else None
    tp = DT.torch_params(g)
    xi = torch.zeros(6, dtype=torch.float64, requires_grad=True)
    C, D, A = DT.render_dense(*tp, sh, cam, torch.tensor(T), xi=xi, sh_signs=signs)
    np.testing.assert_allclose(C.detach().numpy(), out["color"], atol=1e-11)
    np.testing.assert_allclose(D.detach().numpy(), out["depth"], atol=1e-11)
    np.testing.assert_allclose(A.detach().numpy(), out["alpha"], atol=1e-11)
    rng = np.random.default_rng(100 + seed)
    dC = rng.standard_normal(C.shape)
    dD = rng.standard_normal(D.shape)
    dA = rng.standard_normal(A.shape)
    L = (C * torch.tensor(dC)).sum() + (D * torch.tensor(dD)).sum() + (A * torch.tensor(dA)).sum()
    L.backward()
    gr = oracle.backward(g, cam, T, dC, dD, dA)
    names = ["means", "log_scales", "quats", "opacity_logits", "colors"]
    for name, t in zip(names, tp):
        ref = t.grad.numpy()
        err = np.linalg.norm(gr[name] - ref) / max(np.linalg.norm(ref), 1e-30)
        assert err < 1e-9, (name, err)
    err = np.linalg.norm(gr["pose"] - xi.grad.numpy()) / np.linalg.norm(xi.grad.numpy())
    assert err < 1e-9, ("pose", err)


# --------------------------------------------------------------------------
# central finite differences of the oracle itself (FP64)
# --------------------------------------------------------------------------

def _fd_setup(oracle, seed, sh=-1):
    means, ls, q, opl, col, cam, T = _tiny_scene(seed, n=24, W=24, H=20, sh_degree=sh)
    g = oracle.Gaussians(means, ls, q, opl, col, sh)
    wide = oracle.render(g, cam, T, bands=(5e-3, 5e-3, 5e-3))
    rng = np.random.default_rng(seed + 50)
    keep = (wide["ambiguous"] == 0).astype(np.float64)
    dC = rng.standard_normal((3, cam.height, cam.width)) * keep
    dD = rng.standard_normal((cam.height, cam.width)) * keep
    dA = rng.standard_normal((cam.height, cam.width)) * keep
    return g, cam, T, dC, dD, dA


def _loss(oracle, g, cam, T, dC, dD, dA):
    o = oracle.render(g, cam, T)
    return float(np.sum(o["color"] * dC) + np.sum(o["depth"] * dD) + np.sum(o["alpha"] * dA))


@pytest.mark.parametrize("seed,sh", [(4, -1), (5, 2)])
def test_reverse_mode_vs_central_fd(oracle, seed, sh):
    g, cam, T, dC, dD, dA = _fd_setup(oracle, seed, sh)
    gr = oracle.backward(g, cam, T, dC, dD, dA)
    rng = np.random.default_rng(seed)
    for name in ["means", "log_scales", "quats", "opacity_logits", "colors"]:
        arr = getattr(g, name)
        flat = arr.reshape(-1)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            h = 1e-6 * max(1.0, abs(flat[i]))
            old = flat[i]
            flat[i] = old + h
            lp = _loss(oracle, g, cam, T, dC, dD, dA)
            flat[i] = old - h
            lm = _loss(oracle, g, cam, T, dC, dD, dA)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = gr[name].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-7, (name, i, fd, an)
    for k in range(6):
        xi = np.zeros(6)
        xi[k] = 1e-6
        lp = _loss(oracle, g, cam, oracle.se3_exp(xi) @ T, dC, dD, dA)
        lm = _loss(oracle, g, cam, oracle.se3_exp(-xi) @ T, dC, dD, dA)
        fd = (lp - lm) / 2e-6
        assert abs(fd - gr["pose"][k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-7, (k, fd, gr["pose"][k])


def test_single_gaussian_analytic_gradients(oracle):
    """One Gaussian, one pixel: dC/dcolour = alpha and dC/do = colour exp(-sigma)."""
    cam = _cam()
    z, s, opl = 2.0, 0.05, 0.3
    g = _one(oracle, (0.0, 0.0, z), (math.log(s),) * 3, opl=opl)
    pix = np.array([[35, 26]], np.int32)
    out = oracle.render(g, cam, np.eye(4), pixels=pix)
    a = out["alpha"][0]
    dC = np.array([[1.0], [0.0], [0.0]])
    gr = oracle.backward(g, cam, np.eye(4), dC=dC, pixels=pix)
    assert gr["colors"][0, 0] == pytest.approx(a, rel=1e-14)
    o = 1 / (1 + math.exp(-opl))
    # d C_r / d logit = colour_r * exp(-sigma) * o (1 - o) = colour_r * alpha (1 - o)
    assert gr["opacity_logits"][0] == pytest.approx(0.2 * a * (1 - o), rel=1e-12)


# --------------------------------------------------------------------------
# re-projection (Sec. 3.2 Eq. lba) with the Huber kernel
# --------------------------------------------------------------------------

def test_reproj_zero_at_true_pose_and_fd(oracle):
    s = scenes.c4(n=2000, views=3, res_scale=0.25, vis_range=(200, 2000), matches=(50, 80), seed=7)
    cams = s.cams
    # noise-free observations: re-derive the back-projected pixels by
    # re-running the generator without noise is not possible, so build them
    # directly: points at known pixels and depths under the true pose
    rng = np.random.default_rng(0)
    P, U, vid = [], [], []
    for v, c in enumerate(cams):
        px = rng.uniform(0, c.width - 1, 30)
        py = rng.uniform(0, c.height - 1, 30)
        z = rng.uniform(1, 5, 30)
        xc = np.stack([(px - c.cx) / c.fx * z, (py - c.cy) / c.fy * z, z], 1)
        Ti = np.linalg.inv(s.poses_true[v].astype(np.float64))
        P.append(xc @ Ti[:3, :3].T + Ti[:3, 3])
        U.append(np.stack([px, py], 1))
        vid.append(np.full(30, v))
    P, U, vid = np.concatenate(P), np.concatenate(U), np.concatenate(vid).astype(np.int32)
    r = oracle.reproj(cams, s.poses_true.astype(np.float64), P, U, vid, 2.0)
    assert np.abs(r["residual"]).max() < 1e-9
    np.testing.assert_allclose(r["loss"], 0, atol=1e-18)
    # pose gradient vs central FD at the perturbed pose, including outliers
    U2 = U + rng.normal(0, 3.0, U.shape)
    Tp = s.poses.astype(np.float64)
    r = oracle.reproj(cams, Tp, P, U2, vid, 2.0)
    for v in range(len(cams)):
        for k in range(6):
            xi = np.zeros(6)
            xi[k] = 1e-6
            Tpp, Tpm = Tp.copy(), Tp.copy()
            Tpp[v] = oracle.se3_exp(xi) @ Tp[v]
            Tpm[v] = oracle.se3_exp(-xi) @ Tp[v]
            fd = (oracle.reproj(cams, Tpp, P, U2, vid, 2.0)["loss"][v] -
                  oracle.reproj(cams, Tpm, P, U2, vid, 2.0)["loss"][v]) / 2e-6
            assert abs(fd - r["dpose"][v, k]) < 1e-6 * max(1, abs(fd)), (v, k, fd, r["dpose"][v, k])


def test_huber_continuity(oracle):
    """h(e) = e^2/2 for e <= delta, delta (e - delta/2) beyond: value and slope
    continuous at e = delta."""
    cam = scenes.Camera(64, 48, 60, 60, 32, 24)
    P = np.array([[0.0, 0.0, 2.0]] * 3)
    d = 2.0
    U = np.array([[32 + d - 1e-7, 24], [32 + d, 24], [32 + d + 1e-7, 24]])
    r = [oracle.reproj([cam], np.eye(4)[None], P[i:i + 1], U[i:i + 1], np.zeros(1, np.int32), d) for i in range(3)]
    vals = [x["loss"][0] for x in r]
    assert vals[1] == pytest.approx(0.5 * d * d)
    assert abs(vals[0] - vals[1]) < 1e-6 and abs(vals[2] - vals[1]) < 1e-6
    gx = [x["dpose"][0, 0] for x in r]
    assert abs(gx[0] - gx[2]) < 1e-5


def test_reproj_behind_near_plane_excluded(oracle):
    cam = scenes.Camera(64, 48, 60, 60, 32, 24)
    P = np.array([[0.0, 0.0, 0.1], [0.0, 0.0, 2.0]])
    U = np.array([[10.0, 10.0], [33.0, 24.0]])
    r = oracle.reproj([cam], np.eye(4)[None], P, U, np.zeros(2, np.int32), 2.0)
    assert r["nvalid"][0] == 1
    assert r["loss"][0] == pytest.approx(0.5)
    assert np.all(r["residual"][0] == 0)


# --------------------------------------------------------------------------
# binning definition (integer) vs brute force
# --------------------------------------------------------------------------

@pytest.mark.parametrize("tw,th,overhang", [(16, 16, False), (8, 8, False), (32, 8, False), (16, 8, True)])
def test_binning_brute_force(oracle, tw, th, overhang):
    """overhang: rects reaching past their image (up to the 16-bit limit, or
    starting beyond it) bin as their part inside the image; the brute force
    visits only the image's tiles."""
    sizes = [(70, 45), (33, 17), (64, 48)]
    n = 60
    rect, depth = scenes.synthetic_binning_records(sizes, n, seed=tw * 7 + th)
    if overhang:
        rect = rect.copy()
        rng = np.random.default_rng(5)
        for v, (W, H) in enumerate(sizes):
            idx = v * n + rng.choice(n, 20, replace=False)
            rect[idx[:8], 0] = (rect[idx[:8], 0] & 0xFFFF) | (np.uint32(0xFFFF) << 16)
            rect[idx[8:14], 1] = (rect[idx[8:14], 1] & 0xFFFF) | (np.uint32(H + 5) << 16)
            rect[idx[14:], 0] = np.uint32(W + 3) | (np.uint32(W + 9) << 16)
    values, ranges = oracle.binning(sizes, n, tw, th, rect, depth)
    # brute force: per tile, scan every record
    tid = 0
    bits = depth.view(np.uint32)
    for v, (W, H) in enumerate(sizes):
        tx, ty = -(-W // tw), -(-H // th)
        for b in range(ty):
            for a in range(tx):
                lst = []
                # the tile's pixels inside the image
                px0, px1 = a * tw, min((a + 1) * tw, W) - 1
                py0, py1 = b * th, min((b + 1) * th, H) - 1
                for i in range(n):
                    r = v * n + i
                    x0, x1 = int(rect[r, 0] & 0xFFFF), int(rect[r, 0] >> 16)
                    y0, y1 = int(rect[r, 1] & 0xFFFF), int(rect[r, 1] >> 16)
                    # some pixel of the rect is a pixel of the tile
                    if max(x0, px0) <= min(x1, px1) and max(y0, py0) <= min(y1, py1):
                        lst.append((int(bits[r]), r))
                lst.sort()
                s0, s1 = ranges[tid]
                if not lst:
                    assert (s0, s1) == (0, 0)
                else:
                    assert list(values[s0:s1]) == [r for _, r in lst]
                tid += 1
    assert tid == ranges.shape[0]


# --------------------------------------------------------------------------
# SE(3), SH and Adam against library routines
# --------------------------------------------------------------------------

def test_se3_exp_vs_expm(oracle):
    from scipy.linalg import expm
    rng = np.random.default_rng(3)
    for scale in (1e-9, 1e-3, 0.5, 2.5):
        xi = rng.standard_normal(6) * scale
        M = np.zeros((4, 4))
        M[:3, :3] = oracle.hat(xi[3:])
        M[:3, 3] = xi[:3]
        np.testing.assert_allclose(oracle.se3_exp(xi), expm(M), atol=1e-12)
        np.testing.assert_allclose(oracle.se3_exp(xi) @ oracle.se3_exp(-xi), np.eye(4), atol=1e-12)


def test_sh_orthonormal_and_matches_scipy(oracle):
    """Gauss-Legendre x uniform-azimuth quadrature (exact for these degrees):
    the Gram matrix of the 16 basis functions is the identity, and each one
    is (up to sign) the real combination of scipy's complex harmonics."""
    from scipy.special import sph_harm_y
    xg, wg = np.polynomial.legendre.leggauss(12)
    nphi = 24
    phi = 2 * np.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None]).reshape(-1)
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    Y = oracle.sh_basis(3, d)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)
    th = np.arccos(np.clip(ct.reshape(-1), -1, 1))
    pp = ph.reshape(-1)
    for l in range(4):
        for m in range(-l, l + 1):
            c = sph_harm_y(l, abs(m), th, pp)
            if m == 0:
                ref = c.real
            elif m > 0:
                ref = np.sqrt(2) * c.real
            else:
                ref = np.sqrt(2) * c.imag
            got = Y[:, l * l + l + m]
            dot = np.sum(w * got * ref)
            assert abs(abs(dot) - 1) < 1e-10, (l, m, dot)
            np.testing.assert_allclose(got, np.sign(dot) * ref, atol=1e-10)


def test_sh_gradient_fd(oracle):
    rng = np.random.default_rng(4)
    d = rng.standard_normal((10, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y, dY = oracle.sh_basis(3, d, grad=True)
    h = 1e-6
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        fd = (oracle.sh_basis(3, d + e) - oracle.sh_basis(3, d - e)) / (2 * h)
        np.testing.assert_allclose(dY[:, :, j], fd, atol=1e-8)


def test_adam_vs_torch(oracle):
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(20)
    pt = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([pt], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    p = p0.copy()
    m = np.zeros(20)
    v = np.zeros(20)
    for t in range(1, 6):
        g = rng.standard_normal(20)
        pt.grad = torch.tensor(g)
        opt.step()
        dlt, m, v = oracle.adam_step(p, g, m, v, t, 0.01)
        p = p + dlt
        np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-13, atol=1e-15)


# --------------------------------------------------------------------------
# the paper's printed hyper-parameters (Supplementary, Table hyper)
# --------------------------------------------------------------------------

def test_golden_hyperparameters_table():
    with open(os.path.join(GOLDEN, "paper_hyperparams.json")) as f:
        hp = json.load(f)
    v = hp["values"]
    assert (v["alpha"], v["beta"], v["gamma"], v["zeta"], v["tau"]) == (0.75, 20, 0.99, 0.3, 0.005)
    assert (v["w1"], v["w2"], v["w3"], v["w4"], v["w5"]) == (1.5, 0.5, 1, 0.5, 1)


def test_loss_and_upstream_closed_form(oracle):
    """L1 means per view and their sign gradients, with the gate of Sec. 3.3."""
    cams = [scenes.Camera(4, 2, 1, 1, 0, 0), scenes.Camera(2, 2, 1, 1, 0, 0)]
    rng = np.random.default_rng(0)
    P = [8, 4]
    out = {"color": rng.uniform(0, 1, 3 * 12), "depth": rng.uniform(-0.5, 2, 12), "alpha": rng.uniform(0.9, 1, 12)}
    tc = rng.uniform(0, 1, 36)
    td = rng.uniform(-0.5, 2, 12)
    Lc, Ld, dC, dD = oracle.loss_and_upstream(cams, out, tc, td, 1.0, 0.1, gate_gamma=0.95)
    gate = (td > 0) & (out["depth"] > 0) & (out["alpha"] > 0.95)
    # view 1 by hand
    m = gate[8:12]
    ec = out["color"][24:36].reshape(3, 4) - tc[24:36].reshape(3, 4)
    assert Lc[1] == pytest.approx(np.sum(np.abs(ec) * m) / 12)
    assert Ld[1] == pytest.approx(np.sum(np.abs(out["depth"][8:12] - td[8:12]) * m) / 4)
    np.testing.assert_allclose(dD[8:12], 0.1 / 2 / 4 * np.sign(out["depth"][8:12] - td[8:12]) * m)
    assert P == [c.width * c.height for c in cams]


# --------------------------------------------------------------------------
# the discrete branches of the forward model: the 0.99 alpha clamp, the
# termination before T falls below 1e-4, and the Jacobian clamp at 1.3x the
# half field of view (readings of the colour / depth compositing equations,
# Sec. 3.4, and of its local-affine projection, Sec. 3.3-3.4)
# --------------------------------------------------------------------------

def _iso_alpha(cam, u, v, var, o):
    """The paper's isotropic 2D kernel o exp(-|p - mu|^2 / (2 var)) on the
    pixel grid, clamped at 0.99 and cut below 1/255."""
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    f = o * np.exp(-((xs - u) ** 2 + (ys - v) ** 2) / (2 * var))
    f = np.minimum(f, 0.99)
    f[f < 1 / 255] = 0
    return f


def test_alpha_clamp_closed_form(oracle):
    """A wide, nearly opaque Gaussian on the axis: alpha = min(0.99, o e^-sigma)
    exactly, with several pixels at the clamp (the centre pixel reads 0.99,
    not o)."""
    cam = _cam()
    z, s, opl = 2.0, 0.3, 8.0
    col = np.array([0.2, 0.5, 0.9])
    g = _one(oracle, (0.0, 0.0, z), (math.log(s),) * 3, opl=opl, col=col)
    out = oracle.render(g, cam, np.eye(4))
    o = 1 / (1 + math.exp(-opl))
    f = _iso_alpha(cam, cam.cx, cam.cy, (cam.fx * s / z) ** 2 + 0.3, o)
    assert int((f == 0.99).sum()) >= 5
    assert out["alpha"][int(cam.cy), int(cam.cx)] == 0.99
    np.testing.assert_allclose(out["alpha"], f, atol=1e-14)
    np.testing.assert_allclose(out["depth"], z * f, atol=1e-13)
    for k in range(3):
        np.testing.assert_allclose(out["color"][k], col[k] * f, atol=1e-14)


def test_alpha_clamp_reverse_mode_is_flat(oracle):
    """Where the clamp holds, alpha = 0.99 does not move with the opacity, the
    mean or the covariance: d/dparams of (C, A) there is zero except
    dC/dcolour = 0.99, and central differences of the oracle's own forward
    agree (the clamp has a margin of ~1 % at the centre)."""
    cam = _cam()
    z, s, opl = 2.0, 0.3, 8.0
    g = _one(oracle, (0.0, 0.0, z), (math.log(s),) * 3, opl=opl)
    pix = np.array([[int(cam.cx), int(cam.cy)]], np.int32)
    dC = np.array([[1.0], [0.0], [0.0]])
    dA = np.array([1.0])
    gr = oracle.backward(g, cam, np.eye(4), dC=dC, dA=dA, pixels=pix)
    assert gr["colors"][0, 0] == pytest.approx(0.99, rel=1e-15)
    for name in ["means", "log_scales", "quats", "opacity_logits"]:
        assert np.all(gr[name] == 0), name
    assert np.all(gr["pose"] == 0)

    def loss(gg):
        o = oracle.render(gg, cam, np.eye(4), pixels=pix)
        return float(o["color"][0, 0] + o["alpha"][0])

    for name in ["opacity_logits", "means", "log_scales"]:
        arr = getattr(g, name).reshape(-1)
        for i in range(arr.size):
            old = arr[i]
            arr[i] = old + 1e-6
            lp = loss(g)
            arr[i] = old - 1e-6
            lm = loss(g)
            arr[i] = old
            assert abs(lp - lm) / 2e-6 < 1e-9, (name, i)


def _stack(oracle, k, o, zs, cols, s=0.02):
    """k isotropic Gaussians on the optical axis, one behind the other."""
    opl = math.log(o / (1 - o))
    return oracle.Gaussians(np.array([[0.0, 0.0, z] for z in zs]), np.full((k, 3), math.log(s)),
                            np.tile([1.0, 0, 0, 0], (k, 1)), np.full(k, opl), np.asarray(cols, np.float64))


@pytest.mark.parametrize("o,k,m", [(0.85, 8, 4), (0.55, 14, 11), (0.97, 6, 2)])
def test_termination_closed_form(oracle, o, k, m):
    """k Gaussians of opacity o stacked on the axis: at the centre pixel every
    alpha is o, T after n blends is (1 - o)^n, and blending stops before the
    first n with (1 - o)^n < 1e-4, so exactly m are blended.  C, D, A are the
    m-term sums (colour and depth equations; border mask A = 1 - (1 - o)^m)."""
    assert (1 - o) ** m >= 1e-4 * 1.2 and (1 - o) ** (m + 1) < 1e-4 / 1.2   # decisions with margin
    cam = _cam()
    rng = np.random.default_rng(k)
    zs = 2.0 + 0.1 * np.arange(k)
    cols = rng.uniform(0, 1, (k, 3))
    g = _stack(oracle, k, o, zs, cols)
    pix = np.array([[int(cam.cx), int(cam.cy)]], np.int32)
    out = oracle.render(g, cam, np.eye(4), pixels=pix)
    w = o * (1 - o) ** np.arange(m)
    np.testing.assert_allclose(out["color"][:, 0], w @ cols[:m], rtol=1e-13)
    assert out["depth"][0] == pytest.approx(float(w @ zs[:m]), rel=1e-13)
    assert out["alpha"][0] == pytest.approx(1 - (1 - o) ** m, rel=1e-14)
    assert out["tfinal"][0] == pytest.approx((1 - o) ** m, rel=1e-12)
    assert int(out["nblend"][0]) == m
    # the whole image: A never exceeds 1 - 1e-4
    full = oracle.render(g, cam, np.eye(4))
    assert full["alpha"].max() <= 1 - 1e-4


def test_termination_reverse_mode(oracle):
    """Gaussians behind the stop get no gradient at that pixel, the blended
    ones the closed form dA/dlogit_i = o (1 - o) T_final / (1 - o) with
    T_final = (1 - o)^m (product rule on 1 - prod(1 - alpha_j))."""
    cam = _cam()
    o, k, m = 0.85, 8, 4
    zs = 2.0 + 0.1 * np.arange(k)
    g = _stack(oracle, k, o, zs, np.full((k, 3), 0.5))
    pix = np.array([[int(cam.cx), int(cam.cy)]], np.int32)
    gr = oracle.backward(g, cam, np.eye(4), dA=np.array([1.0]), pixels=pix)
    tf = (1 - o) ** m
    np.testing.assert_allclose(gr["opacity_logits"][:m], o * (1 - o) * tf / (1 - o), rtol=1e-12)
    assert np.all(gr["opacity_logits"][m:] == 0)
    assert np.all(gr["means"][m:] == 0) and np.all(gr["log_scales"][m:] == 0)


def _jclamp_scene(oracle, cam, x_over_z, y_over_z, z, s, opl=2.2):
    return _one(oracle, (x_over_z * z, y_over_z * z, z), (math.log(s),) * 3, opl=opl)


@pytest.mark.parametrize("xz,yz", [(0.9, 0.0), (-0.95, 0.1), (0.2, 0.7), (0.78, -0.6)])
def test_jacobian_clamp_closed_form(oracle, xz, yz):
    """An isotropic Gaussian outside the widened field of view (|x/z| > 1.3 W /
    (2 fx) or |y/z| > 1.3 H / (2 fy)) whose footprint still reaches the image:
    its 2D covariance is s^2 J_c J_c^T + 0.3 I with J_c the pinhole Jacobian at
    the clamped point (t_x, t_y, z), t = clamp(x/z) z, while the mean projects
    unclamped.  The render equals the kernel of that covariance."""
    cam = _cam()
    z, s, opl = 2.0, 0.25, 2.2
    limx, limy = 1.3 * cam.width / (2 * cam.fx), 1.3 * cam.height / (2 * cam.fy)
    assert abs(xz) > limx or abs(yz) > limy
    g = _jclamp_scene(oracle, cam, xz, yz, z, s, opl)
    out = oracle.render(g, cam, np.eye(4))
    tx, ty = np.clip(xz, -limx, limx) * z, np.clip(yz, -limy, limy) * z
    f = cam.fx
    Jc = np.array([[f / z, 0, -f * tx / z ** 2], [0, cam.fy / z, -cam.fy * ty / z ** 2]])
    S = s * s * Jc @ Jc.T + 0.3 * np.eye(2)
    Qm = np.linalg.inv(S)
    u, v = f * xz + cam.cx, cam.fy * yz + cam.cy
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    dx, dy = xs - u, ys - v
    sig = 0.5 * (Qm[0, 0] * dx * dx + 2 * Qm[0, 1] * dx * dy + Qm[1, 1] * dy * dy)
    a = np.minimum(1 / (1 + math.exp(-opl)) * np.exp(-sig), 0.99)
    a[a < 1 / 255] = 0
    assert (a > 0).sum() > 20          # the footprint reaches into the image
    np.testing.assert_allclose(out["alpha"], a, atol=1e-13)


def _deep_scene(seed, n=42, W=32, H=24, sh_degree=-1):
    """A tiny scene that takes every discrete branch: a third of the Gaussians
    crowd the image centre at high opacity (alpha clamp, termination), a third
    sit outside the widened field of view with footprints reaching the image
    (Jacobian clamp), the rest as _tiny_scene."""
    rng = np.random.default_rng(seed)
    fx = 30.0
    limx, limy = 1.3 * W / (2 * fx), 1.3 * H / (2 * 31.0)
    k = n // 3
    z1 = rng.uniform(1.5, 3.0, k)
    crowd = np.stack([rng.normal(0, 0.05, k) * z1, rng.normal(0, 0.05, k) * z1, z1], 1)
    z2 = rng.uniform(1.5, 3.0, k)
    sx = rng.choice([-1, 1], k)
    sy = rng.choice([-1, 1], k)
    tx = np.where(rng.uniform(0, 1, k) < 0.6, sx * limx * rng.uniform(1.08, 1.4, k), rng.uniform(-0.3, 0.3, k))
    ty = np.where(np.abs(tx) > limx, rng.uniform(-0.3, 0.3, k), sy * limy * rng.uniform(1.08, 1.4, k))
    outer = np.stack([tx * z2, ty * z2, z2], 1)
    m = n - 2 * k
    z3 = rng.uniform(1.5, 4.0, m)
    rest = np.stack([rng.uniform(-0.6, 0.6, m), rng.uniform(-0.45, 0.45, m), z3], 1)
    # the first three of the crowd are wide and in front: their alpha stays
    # at the 0.99 clamp over a few pixels each
    zf = rng.uniform(1.3, 1.45, 3)
    crowd[:3] = np.stack([np.array([-0.25, 0.0, 0.25]) * zf, rng.uniform(-0.15, 0.15, 3) * zf, zf], 1)
    means = np.concatenate([crowd, outer, rest])
    ls = np.concatenate([rng.normal(-1.3, 0.2, (k, 3)), rng.normal(-1.6, 0.2, (k, 3)), rng.normal(-2.6, 0.4, (m, 3))])
    ls[:3] = rng.normal(-0.6, 0.05, (3, 3))
    q = rng.standard_normal((n, 4))
    opl = np.concatenate([rng.normal(7.0, 1.5, k), rng.normal(1.5, 0.5, k), rng.normal(0.5, 1.0, m)])
    if sh_degree < 0:
        col = rng.uniform(0, 1, (n, 3))
    else:
        K = (sh_degree + 1) ** 2
        col = rng.normal(0, 0.2, (n, K, 3))
        col[:, 0] = rng.uniform(0, 1, (n, 3))
    cam = scenes.Camera(W, H, fx, 31.0, W / 2 - 0.3, H / 2 + 0.2)
    return means, ls, q, opl, col, cam, np.eye(4)


@pytest.mark.parametrize("seed,sh", [(20, -1), (21, 2)])
def test_dense_brute_force_with_every_branch(oracle, seed, sh):
    """The dense torch renderer (clamped Jacobian, alpha clamp and termination
    as masks, gradients by autograd) equals the oracle's forward and reverse
    mode on a scene where each branch is taken many times."""
    means, ls, q, opl, col, cam, T = _deep_scene(seed, sh_degree=sh)
    g = oracle.Gaussians(means, ls, q, opl, col, sh)
    out = oracle.render(g, cam, T, bands=(0, 0, 0, -1.0))
    signs = _sh_signs(oracle, sh) if sh >= 0 else None
    tp = DT.torch_params(g)
    xi = torch.zeros(6, dtype=torch.float64, requires_grad=True)
    st = {}
    C, D, A = DT.render_dense(*tp, sh, cam, torch.tensor(T), xi=xi, sh_signs=signs, stats=st)
    print(st)
    assert st["alpha_clamped"] >= 5 and st["terminated"] >= 10 and st["jclamped_blended"] >= 20, st
    np.testing.assert_allclose(C.detach().numpy(), out["color"], atol=1e-11)
    np.testing.assert_allclose(D.detach().numpy(), out["depth"], atol=1e-11)
    np.testing.assert_allclose(A.detach().numpy(), out["alpha"], atol=1e-11)
    rng = np.random.default_rng(300 + seed)
    dC = rng.standard_normal(C.shape)
    dD = rng.standard_normal(D.shape)
    dA = rng.standard_normal(A.shape)
    L = (C * torch.tensor(dC)).sum() + (D * torch.tensor(dD)).sum() + (A * torch.tensor(dA)).sum()
    L.backward()
    gr = oracle.backward(g, cam, T, dC, dD, dA)
    for name, t in zip(["means", "log_scales", "quats", "opacity_logits", "colors"], tp):
        ref = t.grad.numpy()
        err = np.linalg.norm(gr[name] - ref) / max(np.linalg.norm(ref), 1e-30)
        assert err < 1e-9, (name, err)
    err = np.linalg.norm(gr["pose"] - xi.grad.numpy()) / np.linalg.norm(xi.grad.numpy())
    assert err < 1e-9, ("pose", err)


@pytest.mark.parametrize("seed,sh", [(22, -1), (23, 1)])
def test_reverse_mode_vs_central_fd_every_branch(oracle, seed, sh):
    """Central differences of the oracle's own loss on the branch-heavy scene,
    cotangents zeroed where a decision sits within the FD step of a threshold
    (the clamped Jacobian has a margin of >= 8 % by construction)."""
    means, ls, q, opl, col, cam, T = _deep_scene(seed, n=30, W=24, H=20, sh_degree=sh)
    g = oracle.Gaussians(means, ls, q, opl, col, sh)
    wide = oracle.render(g, cam, T, bands=(5e-3, 5e-3, 5e-3))
    rng = np.random.default_rng(seed + 50)
    keep = (wide["ambiguous"] == 0).astype(np.float64)
    dC = rng.standard_normal((3, cam.height, cam.width)) * keep
    dD = rng.standard_normal((cam.height, cam.width)) * keep
    dA = rng.standard_normal((cam.height, cam.width)) * keep
    gr = oracle.backward(g, cam, T, dC, dD, dA)
    n = means.shape[0]
    k = n // 3
    # every parameter of the clamped-Jacobian Gaussians, a sample of the rest
    checks = []
    for name, width in [("means", 3), ("log_scales", 3), ("quats", 4), ("opacity_logits", 1)]:
        for i in range(k, 2 * k):
            for j in range(width):
                checks.append((name, i * width + j))
        for i in rng.choice(n, 4, replace=False):
            checks.append((name, int(i) * width))
    for name, idx in checks:
        flat = getattr(g, name).reshape(-1)
        h = 1e-6 * max(1.0, abs(flat[idx]))
        old = flat[idx]
        flat[idx] = old + h
        lp = _loss(oracle, g, cam, T, dC, dD, dA)
        flat[idx] = old - h
        lm = _loss(oracle, g, cam, T, dC, dD, dA)
        flat[idx] = old
        fd = (lp - lm) / (2 * h)
        an = gr[name].reshape(-1)[idx]
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-7, (name, idx, fd, an)
    for j in range(6):
        xi = np.zeros(6)
        xi[j] = 1e-6
        lp = _loss(oracle, g, cam, oracle.se3_exp(xi) @ T, dC, dD, dA)
        lm = _loss(oracle, g, cam, oracle.se3_exp(-xi) @ T, dC, dD, dA)
        fd = (lp - lm) / 2e-6
        assert abs(fd - gr["pose"][j]) <= 1e-6 * max(1.0, abs(fd)) + 1e-7, (j, fd, gr["pose"][j])


def test_se3_left_jacobian_vs_expm_logm(oracle):
    """J_l(xi) e = Log(Exp(xi + e) Exp(xi)^-1) to first order: central
    differences of scipy's matrix exponential and logarithm.  Also J_l(0) = I
    and J_l(xi) xi = xi (ad(xi) xi = 0)."""
    from scipy.linalg import expm, logm
    rng = np.random.default_rng(8)

    def hat6(x):
        M = np.zeros((4, 4))
        M[:3, :3] = oracle.hat(x[3:])
        M[:3, 3] = x[:3]
        return M

    def vee(M):
        return np.array([M[0, 3], M[1, 3], M[2, 3], M[2, 1], M[0, 2], M[1, 0]])

    np.testing.assert_allclose(oracle.se3_left_jacobian(np.zeros(6)), np.eye(6), atol=0)
    for scale in (1e-3, 0.3, 1.2):
        xi = rng.standard_normal(6) * scale
        J = oracle.se3_left_jacobian(xi)
        np.testing.assert_allclose(J @ xi, xi, atol=1e-13)
        Einv = expm(-hat6(xi))
        h = 1e-6
        Jn = np.zeros((6, 6))
        for k in range(6):
            e = np.zeros(6)
            e[k] = h
            lp = vee(np.real(logm(expm(hat6(xi + e)) @ Einv)))
            lm = vee(np.real(logm(expm(hat6(xi - e)) @ Einv)))
            Jn[:, k] = (lp - lm) / (2 * h)
        np.testing.assert_allclose(J, Jn, atol=1e-7)


# --------------------------------------------------------------------------
# blend-order ties: the bound on what reordering near-tied Gaussians changes
# --------------------------------------------------------------------------

def _tied(oracle, zs, cols, opls, scales):
    k = len(zs)
    return oracle.Gaussians(np.array([[0.0, 0.0, z] for z in zs]), np.log(np.array(scales))[:, None] * np.ones((1, 3)),
                            np.tile([1.0, 0, 0, 0], (k, 1)), np.array(opls, float), np.array(cols, float))


def test_order_bound_exact_for_a_swapped_pair(oracle):
    """Two Gaussians whose depths differ by 1e-7 relative (within FP32
    rounding of a depth): swapping which is nearer changes C by exactly
    a1 a2 |c1 - c2| (T0 = 1), which is the oracle's bound, up to the 1e-7
    change of the footprints."""
    cam = _cam()
    z = 2.0
    cols = [[0.9, 0.1, 0.3], [0.2, 0.7, 0.5]]
    a = _tied(oracle, [z, z * (1 + 1e-7)], cols, [0.4, 1.1], [0.05, 0.07])
    b = _tied(oracle, [z * (1 + 1e-7), z], cols, [0.4, 1.1], [0.05, 0.07])
    ra, rb = oracle.render(a, cam, np.eye(4)), oracle.render(b, cam, np.eye(4))
    both = (ra["nblend"] == 2)
    assert both.sum() > 20
    assert np.all(ra["ambiguous"][both] & oracle.AMB_ORDER)
    dC = np.abs(ra["color"] - rb["color"])[:, both]
    bound = ra["order_bound"][:3, both]
    # moving a depth by 1e-7 relative moves its footprint's alpha by at most
    # ~1e-6 alpha (sigma <= ln(255 o) inside the support)
    np.testing.assert_allclose(dC, bound, rtol=1e-5, atol=2e-6)
    # alpha does not depend on the order
    np.testing.assert_allclose(ra["alpha"], rb["alpha"], rtol=0, atol=2e-6)
    # pixels with one Gaussian or none carry no bound
    assert np.all(ra["order_bound"][:, ~both] == 0)


def test_order_bound_covers_every_permutation_of_a_triple(oracle):
    import itertools
    cam = _cam()
    z = 3.0
    cols = [[0.9, 0.1, 0.3], [0.2, 0.7, 0.5], [0.5, 0.5, 0.95]]
    opls, scales = [0.2, 1.5, -0.3], [0.06, 0.05, 0.08]
    eps = [0.0, 0.8e-7, 1.6e-7]
    base = oracle.render(_tied(oracle, [z * (1 + e) for e in eps], cols, opls, scales), cam, np.eye(4))
    three = base["nblend"] == 3
    assert three.sum() > 20
    worst = np.zeros(3)
    for perm in itertools.permutations(range(3)):
        zs = [z * (1 + eps[perm[i]]) for i in range(3)]
        r = oracle.render(_tied(oracle, zs, cols, opls, scales), cam, np.eye(4))
        d = np.abs(r["color"] - base["color"])[:, three]
        assert np.all(d <= base["order_bound"][:3, three] * (1 + 1e-5) + 2e-6)
        worst = np.maximum(worst, (d / np.maximum(base["order_bound"][:3, three], 1e-30)).max(axis=1))
    print("largest change / bound per channel:", worst)


def test_order_bound_at_the_stop(oracle):
    """A tied pair straddling the stop: an opaque front Gaussian (T = 0.05
    behind it), then two Gaussians at depths 1e-7 apart with opacities 0.9
    and 0.99.  In one order the 0.9 one blends (T = 5e-3) and the 0.99 one
    stops the pixel; in the other the 0.99 one blends (T = 5e-4) and the 0.9
    one stops it.  Colour, depth and alpha move by less than the oracle's
    bound (T0 times the largest colour / depth, T0 for alpha, T0 = 0.05)."""
    cam = _cam()
    cols = [[0.1, 0.2, 0.3], [0.9, 0.1, 0.5], [0.2, 0.8, 0.6]]
    ops = [0.95, 0.9, 0.99]
    opl = [math.log(o / (1 - o)) for o in ops]
    sc = [0.02, 0.02, 0.02]
    z2 = 2.2
    pix = np.array([[int(cam.cx), int(cam.cy)]], np.int32)
    a = oracle.render(_tied(oracle, [2.0, z2, z2 * (1 + 1e-7)], cols, opl, sc), cam, np.eye(4), pixels=pix)
    b = oracle.render(_tied(oracle, [2.0, z2 * (1 + 1e-7), z2], cols, opl, sc), cam, np.eye(4), pixels=pix)
    assert a["ambiguous"][0] & oracle.AMB_ORDER_STOP and b["ambiguous"][0] & oracle.AMB_ORDER_STOP
    assert int(a["nblend"][0]) == 2 and int(b["nblend"][0]) == 2
    T0 = 1 - 0.95
    np.testing.assert_allclose(a["tfinal"][0], T0 * (1 - 0.9), rtol=1e-6)
    np.testing.assert_allclose(b["tfinal"][0], T0 * (1 - 0.99), rtol=1e-5)
    bnd = a["order_bound"][:, 0]
    np.testing.assert_allclose(bnd[:3], T0 * np.max(cols[1:], axis=0), rtol=1e-6)
    np.testing.assert_allclose(bnd[4], T0, rtol=1e-12)
    assert np.all(np.abs(a["color"][:, 0] - b["color"][:, 0]) <= bnd[:3])
    assert abs(a["depth"][0] - b["depth"][0]) <= bnd[3]
    assert abs(a["alpha"][0] - b["alpha"][0]) <= bnd[4]
