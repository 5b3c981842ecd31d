"""Pins of the oracle's eight-parameter isotropic Gaussian (Sec. 3.4
"Gaussian Representation", Eq. gauss; projection equation; Eq. d).

The oracle maps the paper's parameters (centre, one log radius, opacity
logit, colour) onto the anisotropic ones with equal scales; these tests
check that map against the paper's closed forms and against finite
differences of the oracle's own forward pass.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from synth import scenes


def _cam(W=64, H=48, f=60.0, cx=32.0, cy=24.0):
    return scenes.Camera(W, H, f, f, cx, cy)


def _pose(rng, p_cam):
    """A random world-to-camera pose and the world point it maps to p_cam."""
    T = np.eye(4)
    T[:3, :3] = Rotation.from_rotvec(rng.normal(0, 0.6, 3)).as_matrix()
    T[:3, 3] = rng.normal(0, 0.5, 3)
    mu = T[:3, :3].T @ (np.asarray(p_cam, float) - T[:3, 3])
    return T, mu


@pytest.mark.parametrize("z,r", [(2.0, 0.05), (3.5, 0.02), (0.9, 0.004)])
def test_isotropic_parameters_project_to_the_paper_radius(oracle, z, r):
    """On the optical axis of any camera pose the footprint is the paper's
    r2D = f r / d: 2D covariance (f r / d)^2 I plus the 0.3 px^2 dilation."""
    cam = _cam()
    rng = np.random.default_rng(int(z * 100))
    T, mu = _pose(rng, (0.0, 0.0, z))
    g = oracle.from_isotropic(mu[None], [math.log(r)], [1.5], [[0.1, 0.2, 0.3]])
    rec = oracle.project(g, cam, T)[0]
    r2d = cam.fx * r / z
    assert rec[0] == 1
    assert rec[1] == pytest.approx(cam.cx, abs=1e-9) and rec[2] == pytest.approx(cam.cy, abs=1e-9)
    assert rec[16] - 0.3 == pytest.approx(r2d ** 2, rel=1e-10)
    assert rec[18] - 0.3 == pytest.approx(r2d ** 2, rel=1e-10)
    assert abs(rec[17]) < 1e-10 * r2d ** 2


@pytest.mark.parametrize("p", [(0.4, -0.3, 2.0), (-0.9, 0.6, 1.6), (0.05, 0.7, 3.0)])
def test_isotropic_off_axis_covariance_closed_form(oracle, p):
    """Off the axis the local affine footprint of the covariance r^2 I is
    r^2 J J^T with the pinhole Jacobian J = [[f/z, 0, -f x/z^2], [0, f/z,
    -f y/z^2]] at the camera point, whatever the camera's rotation."""
    cam = _cam()
    rng = np.random.default_rng(7)
    r = 0.03
    T, mu = _pose(rng, p)
    g = oracle.from_isotropic(mu[None], [math.log(r)], [0.5], [[0.5, 0.5, 0.5]])
    rec = oracle.project(g, cam, T)[0]
    x, y, z = p
    f = cam.fx
    J = np.array([[f / z, 0.0, -f * x / z ** 2], [0.0, f / z, -f * y / z ** 2]])
    S = r * r * J @ J.T
    assert rec[0] == 1
    np.testing.assert_allclose([rec[16] - 0.3, rec[17], rec[18] - 0.3], [S[0, 0], S[0, 1], S[1, 1]], rtol=1e-9,
                               atol=1e-12)
    np.testing.assert_allclose([rec[1], rec[2]], [f * x / z + cam.cx, f * y / z + cam.cy], rtol=1e-12)


def _iso_scene(seed, n=24, W=24, H=20):
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-0.6, 0.6, n), rng.uniform(-0.45, 0.45, n), rng.uniform(1.5, 4.0, n)], 1)
    lr = rng.normal(-2.5, 0.4, n)
    opl = rng.normal(0.5, 1.0, n)
    col = rng.uniform(0, 1, (n, 3))
    cam = scenes.Camera(W, H, 30.0, 31.0, W / 2 - 0.3, H / 2 + 0.2)
    T = np.eye(4)
    T[:3, :3] = Rotation.from_rotvec(rng.normal(0, 0.05, 3)).as_matrix()
    T[:3, 3] = rng.normal(0, 0.05, 3)
    return means, lr, opl, col, cam, T


@pytest.mark.parametrize("seed", [3, 8])
def test_isotropic_reverse_mode_vs_central_fd(oracle, seed):
    """Central differences in the eight parameters themselves (the log radius
    moves all three scales at once) against the oracle's reverse mode mapped
    by isotropic_grads."""
    means, lr, opl, col, cam, T = _iso_scene(seed)
    wide = oracle.render(oracle.from_isotropic(means, lr, opl, col), cam, T, bands=(5e-3, 5e-3, 5e-3))
    rng = np.random.default_rng(seed + 1)
    keep = (wide["ambiguous"] == 0).astype(np.float64)
    dC = rng.standard_normal((3, cam.height, cam.width)) * keep
    dD = rng.standard_normal((cam.height, cam.width)) * keep
    dA = rng.standard_normal((cam.height, cam.width)) * keep

    def loss():
        o = oracle.render(oracle.from_isotropic(means, lr, opl, col), cam, T)
        return float(np.sum(o["color"] * dC) + np.sum(o["depth"] * dD) + np.sum(o["alpha"] * dA))

    gr = oracle.isotropic_grads(oracle.backward(oracle.from_isotropic(means, lr, opl, col), cam, T, dC, dD, dA))
    assert set(gr) == {"means", "log_radius", "opacity_logits", "colors", "pose"}
    assert gr["log_radius"].shape == lr.shape
    checked = 0
    for name, arr in [("log_radius", lr), ("means", means), ("opacity_logits", opl), ("colors", col)]:
        flat = arr.reshape(-1)
        for i in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            h = 1e-6 * max(1.0, abs(flat[i]))
            old = flat[i]
            flat[i] = old + h
            lp = loss()
            flat[i] = old - h
            lm = loss()
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = gr[name].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-7, (name, i, fd, an)
            checked += abs(an) > 1e-3
    assert checked >= 10      # the scene is not trivially flat


def test_isotropic_densify_gives_one_pixel_footprints(oracle):
    """Eq. d with the isotropic parameters: every Gaussian densification adds
    (radius d / f) projects, in the view it came from, to a footprint whose
    smaller principal variance is exactly 1 px^2 (f r / d = 1 across the
    viewing ray; the other axis is stretched by the pinhole obliquity)."""
    cam = _cam(W=20, H=14, f=40.0, cx=9.7, cy=7.2)
    rng = np.random.default_rng(11)
    T, _ = _pose(rng, (0.0, 0.0, 1.0))
    P = cam.width * cam.height
    depth = rng.uniform(0.8, 3.0, P)
    depth[rng.random(P) < 0.2] = 0.0
    col = rng.random(3 * P)
    alpha = rng.random(P)
    new, where = oracle.densify([cam], [T], alpha, col, depth, 0.5, False, isotropic=True)
    assert set(new) == {"means", "log_radius", "opacity_logits", "colors"}
    assert len(where) == int(((depth > 0) & (alpha <= 0.5)).sum()) > 20
    g = oracle.from_isotropic(new["means"], new["log_radius"], np.full(len(where), 2.0), new["colors"])
    rec = oracle.project(g, cam, T)
    assert rec[:, 0].all()
    np.testing.assert_allclose(rec[:, 1], where[:, 1], atol=1e-9)
    np.testing.assert_allclose(rec[:, 2], where[:, 2], atol=1e-9)
    for a, b, c in rec[:, 16:19]:
        S = np.array([[a - 0.3, b], [b, c - 0.3]])
        assert np.linalg.eigvalsh(S)[0] == pytest.approx(1.0, rel=1e-9)


def test_isotropic_adam_layout_has_eight_floats_per_gaussian(oracle):
    """Sec. 3.4: eight parameters per Gaussian (3 colour, 3 centre, 1 radius,
    1 opacity), so the Adam moments hold 8 floats per RGB Gaussian (14 for
    the anisotropic form) before the 6 per view of the poses."""
    groups, pose = oracle.adam_groups(1000, -1, 4, isotropic=True)
    assert pose == 8 * 1000 and [w for _, w in groups] == [3, 1, 0, 1, 3]
    assert oracle.adam_groups(1000, -1, 4)[1] == 14 * 1000
    assert oracle.adam_groups(10, 3, 2, isotropic=True)[1] == (5 + 48) * 10
