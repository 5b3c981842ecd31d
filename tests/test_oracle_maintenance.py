"""Pins of the oracle's map maintenance (Sec. 3.4 pruning and densification)
against brute force, the oracle's own projection code and closed forms."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from synth import scenes


def _params(n, seed, sh=-1):
    rng = np.random.default_rng(seed)
    K = 1 if sh < 0 else (sh + 1) ** 2
    return {"means": rng.standard_normal((n, 3)), "log_scales": rng.standard_normal((n, 3)) - 3,
            "quats": rng.standard_normal((n, 4)), "opacity_logits": rng.standard_normal(n) * 3,
            "colors": rng.random((n, 3)) if sh < 0 else rng.standard_normal((n, K, 3))}


def test_prune_matches_brute_force():
    p = _params(500, 1)
    tau = 0.2
    kept, idx = O.prune(p, tau)
    want = [i for i in range(500) if not (1.0 / (1.0 + math.exp(-p["opacity_logits"][i])) < tau)]
    assert list(idx) == want
    for k in p:
        np.testing.assert_array_equal(kept[k], np.asarray(p[k])[want])


def test_prune_limits_and_idempotence():
    p = _params(300, 2)
    assert len(O.prune(p, 0.0)[1]) == 300            # opacity is never negative
    assert len(O.prune(p, 1.0 + 1e-9)[1]) == 0        # nor above one
    kept, _ = O.prune(p, 0.005)
    again, idx = O.prune(kept, 0.005)
    assert len(idx) == len(kept["opacity_logits"])


def _rgbd(cams, seed):
    rng = np.random.default_rng(seed)
    P = sum(c.width * c.height for c in cams)
    depth = rng.uniform(0.5, 4.0, P)
    depth[rng.random(P) < 0.1] = 0.0                  # holes in the sensor depth
    return rng.random(3 * P), depth, rng.random(P)


def test_densify_selection_matches_mask_count():
    cams = [scenes.Camera(9, 7, 8.0, 8.0, 4.0, 3.0), scenes.Camera(5, 6, 5.0, 6.0, 2.0, 3.0)]
    poses = [np.eye(4), O.se3_exp([0.1, -0.2, 0.05, 0.1, 0.0, -0.2])]
    col, dep, alpha = _rgbd(cams, 3)
    for all_px, gamma in [(True, 0.99), (False, 0.5), (False, 0.99)]:
        new, where = O.densify(cams, poses, alpha, col, dep, gamma, all_px)
        sel = (dep > 0) & (True if all_px else (alpha <= gamma))
        assert len(where) == int(np.sum(sel))
        flat = np.concatenate([np.arange(c.width * c.height) for c in cams])
        view = np.concatenate([np.full(c.width * c.height, v) for v, c in enumerate(cams)])
        assert [tuple(w) for w in where] == [(int(view[i]), int(flat[i] % cams[view[i]].width),
                                              int(flat[i] // cams[view[i]].width)) for i in np.nonzero(sel)[0]]


@pytest.mark.parametrize("sh", [-1, 2])
def test_densified_gaussians_land_on_their_pixels(sh):
    """Projected by the oracle's C projection, every new Gaussian sits at its
    pixel's sample point at the sensor depth, shows the target colour, and on
    the optical axis its footprint is one pixel (sigma^2 = 1, plus the 0.3 px^2
    dilation)."""
    cam = scenes.Camera(11, 9, 10.0, 10.0, 5.0, 4.0)
    T = O.se3_exp([0.2, 0.1, -0.3, 0.05, -0.1, 0.02])
    col, dep, alpha = _rgbd([cam], 4)
    new, where = O.densify([cam], [T], alpha, col, dep, 0.99, True, sh_degree=sh)
    g = O.Gaussians(new["means"], new["log_scales"], new["quats"], new["opacity_logits"], new["colors"], sh)
    rec = O.project(g, cam, T)
    P = cam.width * cam.height
    for i, (_, x, y) in enumerate(where):
        assert rec[i, 0] == 1.0
        assert abs(rec[i, 1] - x) < 1e-9 and abs(rec[i, 2] - y) < 1e-9
        assert abs(rec[i, 10] - dep[y * cam.width + x]) < 1e-9
        assert abs(rec[i, 6] - 0.5) < 1e-15
        np.testing.assert_allclose(rec[i, 7:10], col[[y * cam.width + x, P + y * cam.width + x,
                                                      2 * P + y * cam.width + x]], rtol=0, atol=1e-12)
        if x == 5 and y == 4:
            np.testing.assert_allclose(rec[i, 16:19], [1.3, 0.0, 1.3], atol=1e-12)


def test_adam_relayout():
    n, sh, V = 7, 1, 2
    groups, pose_off = O.adam_groups(n, sh, V)
    m = np.arange(pose_off + 6 * V, dtype=np.float64)
    src = np.array([6, 0, 3, -1, -1])
    out = O.adam_relayout(m, n, sh, V, src, 5)
    new_groups, new_pose = O.adam_groups(5, sh, V)
    for (oo, w), (on, _) in zip(groups, new_groups):
        for i, j in enumerate(src):
            for e in range(w):
                want = 0.0 if j < 0 else m[oo + w * j + e]
                assert out[on + w * i + e] == want
    np.testing.assert_array_equal(out[new_pose:], m[pose_off:])


def test_point_gradients_match_central_differences():
    """The oracle's point gradient against central differences of the C
    oracle's re-projection loss (independent code)."""
    rng = np.random.default_rng(12)
    cams = [scenes.Camera(64, 48, 60.0, 60.0, 32.0, 24.0), scenes.Camera(40, 30, 35.0, 35.0, 20.0, 15.0)]
    poses = [np.eye(4), O.se3_exp([0.1, 0.0, 0.05, 0.02, -0.03, 0.01])]
    M = 12
    P = np.column_stack([rng.uniform(-1, 1, M), rng.uniform(-1, 1, M), rng.uniform(2, 4, M)])
    vid = (np.arange(M) % 2).astype(np.int32)
    U = np.zeros((M, 2))
    for m in range(M):
        T = poses[vid[m]]
        p = T[:3, :3] @ P[m] + T[:3, 3]
        c = cams[vid[m]]
        U[m] = [c.fx * p[0] / p[2] + c.cx, c.fy * p[1] / p[2] + c.cy]
    U += rng.normal(0, 1.5, U.shape)      # some residuals beyond the Huber knee
    g = O.reproj_point_grads(cams, poses, P, U, vid, 2.0, weight=0.7)

    def loss(Pm):
        return 0.7 * float(O.reproj(cams, poses, Pm, U, vid, 2.0)["loss"].sum())

    h = 1e-6
    for m in range(M):
        for k in range(3):
            e = np.zeros_like(P)
            e[m, k] = h
            fd = (loss(P + e) - loss(P - e)) / (2 * h)
            assert abs(fd - g[m, k]) <= 1e-6 * max(1.0, abs(fd)), (m, k, fd, g[m, k])


def test_viewpoint_selection_worked_example():
    """A hand-worked sequence (alpha = 0.75, beta = 20): keyframe 1 shares 100
    of the 120 points of keyframe 0 (>= 0.75 * 120 = 90: too similar), keyframe
    2 shares 60 (selected), keyframe 3 shares 10 with keyframe 2 (< 20: too
    few), keyframe 4 shares 30 with keyframe 2 (selected: 30 < 0.75 * 80)."""
    covis = np.zeros((5, 5), np.int32)
    covis[0, 1], covis[0, 2], covis[2, 3], covis[2, 4] = 100, 60, 10, 30
    n_obs = np.array([120, 110, 80, 70, 90], np.int32)
    assert list(O.select_viewpoints(covis, n_obs, 0.75, 20)) == [True, False, True, False, True]
