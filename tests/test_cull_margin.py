"""The forward projection first culls (Gaussian, view) pairs with a cheap
conservative test and fully projects only the pairs that pass; a pair the
full projection would give a non-empty pixel rect must never be culled.
The test bounds the 2D covariance's diagonal by the largest scale squared
times |J W|^2, widens it (1 % plus 0.01 px^2, the half-width by 0.1 % plus
0.01 px, the near plane by 0.1 %, the image by one pixel) and uses the
hardware reciprocal and square root (about one ulp).  This emulates both
sides in FP32 over random poses (non-rigid ones included), scales over
several decades, and opacities around the threshold, with the cull's
reciprocal and square roots perturbed by four ulps in either direction, and
checks that no accepted pair is culled.  A companion check shows that the
comparison catches a non-conservative bound (the smallest scale in place of
the largest)."""
import numpy as np

F = np.float32
Z_NEAR = F(0.2)
J_CLAMP = F(1.3)
DILATE = F(0.3)


def _rot(q):
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                  2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                  2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1)
    return R.reshape(-1, 3, 3).astype(F)


def _pose(rng, nonrigid):
    """World-to-camera 3x4 (rotation from a random axis-angle, optionally
    scaled per axis), FP32."""
    ax = rng.normal(0.0, 1.0, 3)
    th = np.linalg.norm(ax)
    k = ax / th
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    R = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K
    if nonrigid:
        R = R @ np.diag(rng.uniform(0.5, 2.0, 3))
    T = np.zeros((3, 4))
    T[:, :3] = R
    T[:, 3] = rng.normal(0.0, 1.0, 3)
    return T.astype(F)


def _accepted(p, Sc, o, W, H, fx, fy, cx, cy):
    """The full projection's verdict: near plane, positive 2D covariance,
    opacity above 1/255 and a non-empty pixel rect (bounding box of the
    alpha ellipse at the widened level, capped by the radius)."""
    pz = p[:, 2]
    ok = pz > Z_NEAR
    iz = (F(1) / np.where(ok, pz, F(1))).astype(F)
    u = (fx * p[:, 0] * iz + cx).astype(F)
    v = (fy * p[:, 1] * iz + cy).astype(F)
    limx = J_CLAMP * F(W) / (F(2) * fx)
    limy = J_CLAMP * F(H) / (F(2) * fy)
    tx = (np.clip(p[:, 0] * iz, -limx, limx) * pz).astype(F)
    ty = (np.clip(p[:, 1] * iz, -limy, limy) * pz).astype(F)
    n = p.shape[0]
    J = np.zeros((n, 2, 3), F)
    J[:, 0, 0] = fx * iz
    J[:, 0, 2] = -fx * tx * iz * iz
    J[:, 1, 1] = fy * iz
    J[:, 1, 2] = -fy * ty * iz * iz
    S2 = np.einsum("nij,njk,nlk->nil", J, Sc, J).astype(F)
    a = S2[:, 0, 0] + DILATE
    b = S2[:, 0, 1]
    c = S2[:, 1, 1] + DILATE
    det = a * c - b * b
    with np.errstate(divide="ignore", invalid="ignore"):
        qbox = (F(2) * np.log(F(255) * o)).astype(F) + F(0.05)
        m = F(0.5) * (a + c)
        lmax = m + np.sqrt(np.maximum(m * m - det, 0)).astype(F)
        r = np.ceil(np.sqrt(np.maximum(qbox * lmax, 0)))
        hx = np.minimum(r, np.sqrt(np.maximum(qbox * a, 0)) + F(0.01))
        hy = np.minimum(r, np.sqrt(np.maximum(qbox * c, 0)) + F(0.01))
    x0 = np.maximum(np.ceil(u - hx), 0)
    x1 = np.minimum(np.floor(u + hx), W - 1)
    y0 = np.maximum(np.ceil(v - hy), 0)
    y1 = np.minimum(np.floor(v + hy), H - 1)
    return ok & (det > 0) & (o >= F(1 / 255)) & (x0 <= x1) & (y0 <= y1)


def _cull_passes(p, Wr, smax2, o, W, H, fx, fy, cx, cy, d_rcp, d_sqrt):
    """The cheap test with the reciprocal scaled by (1 + d_rcp) and both
    square roots by (1 + d_sqrt)."""
    pz = p[:, 2]
    iz = ((F(1) / np.where(pz > 0, pz, F(1))) * F(1 + d_rcp)).astype(F)
    u = (fx * p[:, 0] * iz + cx).astype(F)
    v = (fy * p[:, 1] * iz + cy).astype(F)
    limx = J_CLAMP * F(W) / (F(2) * fx)
    limy = J_CLAMP * F(H) / (F(2) * fy)
    tx = (np.clip(p[:, 0] * iz, -limx, limx) * pz).astype(F)
    ty = (np.clip(p[:, 1] * iz, -limy, limy) * pz).astype(F)
    j00, j11 = fx * iz, fy * iz
    j02, j12 = -fx * tx * iz * iz, -fy * ty * iz * iz
    wx = j00[:, None] * Wr[0] + j02[:, None] * Wr[2]
    wy = j11[:, None] * Wr[1] + j12[:, None] * Wr[2]
    a = F(1.01) * (wx * wx).sum(1) * smax2 + (DILATE + F(0.01))
    c = F(1.01) * (wy * wy).sum(1) * smax2 + (DILATE + F(0.01))
    with np.errstate(divide="ignore", invalid="ignore"):
        qbox = np.where(o >= F(1 / 255), (F(2) * np.log(F(255) * o)).astype(F) + F(0.05), F(-1))
        s = F(1 + d_sqrt)
        hx = F(1.001) * (np.sqrt(qbox * a) * s).astype(F) + F(0.02)
        hy = F(1.001) * (np.sqrt(qbox * c) * s).astype(F) + F(0.02)
    return (pz > F(0.999) * Z_NEAR) & (qbox > 0) & (u + hx >= -1) & (u - hx <= W) & (v + hy >= -1) & (v - hy <= H)


def _scene(rng, trial, n):
    W, H = [(1200, 680), (640, 480), (64, 48), (33, 17)][trial % 4]
    fx = fy = F(W * 0.5 * rng.uniform(0.6, 1.6))
    cx, cy = F(W / 2), F(H / 2)
    T = _pose(rng, nonrigid=trial % 5 == 4)
    mu = rng.uniform(-6, 6, (n, 3)).astype(F)
    ls = rng.normal(-2.5, 1.5, (n, 3)).astype(F)
    if trial % 3 == 0:
        ls[:] = ls[:, :1]
    s = np.exp(ls).astype(F)
    R = _rot(rng.standard_normal((n, 4)))
    o = (1 / (1 + np.exp(-rng.normal(0, 3, n)))).astype(F)
    M = np.einsum("nij,nj,nkj->nik", R, s * s, R).astype(F)
    p = (mu @ T[:, :3].T + T[:, 3]).astype(F)
    Wr = T[:, :3]
    Sc = np.einsum("ij,njk,lk->nil", Wr, M, Wr).astype(F)
    return p, Wr, Sc, s, o, W, H, fx, fy, cx, cy


def test_cull_never_drops_an_accepted_pair():
    rng = np.random.default_rng(5)
    accepted = passed = 0
    for trial in range(20):
        p, Wr, Sc, s, o, W, H, fx, fy, cx, cy = _scene(rng, trial, 40000)
        smax2 = (s.max(1) ** 2).astype(F)
        acc = _accepted(p, Sc, o, W, H, fx, fy, cx, cy)
        ulp4 = 2.0 ** -21
        cull = np.ones_like(acc)
        for d_rcp in (-ulp4, ulp4):
            cull &= _cull_passes(p, Wr, smax2, o, W, H, fx, fy, cx, cy, d_rcp, -ulp4)
        missed = acc & ~cull
        assert not missed.any(), (trial, np.nonzero(missed)[0][:5])
        accepted += int(acc.sum())
        passed += int(cull.sum())
    assert accepted > 10000
    # the bound is loose by design but not wildly so
    assert passed <= 2 * accepted, (passed, accepted)


def test_check_catches_a_non_conservative_bound():
    """The same comparison with the smallest scale squared in place of the
    largest (a plausible slip) finds culled pairs that the full projection
    accepts, so the check above can fail."""
    rng = np.random.default_rng(6)
    dropped = 0
    for trial in range(8):
        p, Wr, Sc, s, o, W, H, fx, fy, cx, cy = _scene(rng, trial, 40000)
        acc = _accepted(p, Sc, o, W, H, fx, fy, cx, cy)
        smin2 = (s.min(1) ** 2).astype(F)
        wrong = _cull_passes(p, Wr, smin2, o, W, H, fx, fy, cx, cy, 0.0, 0.0)
        dropped += int((acc & ~wrong).sum())
    assert dropped > 0
