"""The compositing kernels test no support rect per pixel: a pixel outside a
record's rect must have an exact alpha at least 2.5 % below the 1/255
threshold, so that the alpha test alone rejects it (far above FP32 rounding).
This pins that property of the rect construction (bounding box of the
ellipse at the widened level q = 2 ln(255 o) + 0.05, plus 0.01 px, capped by
ceil(sqrt(q lambda_max))) in FP64 over random 2D footprints, including
elongated and rotated ones and opacities near the threshold."""
import numpy as np


def _rect_halfwidths(a, b, c, o):
    q = 2.0 * np.log(255.0 * o) + 0.05
    m = 0.5 * (a + c)
    lmax = m + np.sqrt(np.maximum(m * m - (a * c - b * b), 0.0))
    r = np.ceil(np.sqrt(q * lmax))
    return np.minimum(r, np.sqrt(q * a) + 0.01), np.minimum(r, np.sqrt(q * c) + 0.01)


def test_alpha_outside_rect_is_below_threshold_with_margin():
    rng = np.random.default_rng(7)
    n = 4000
    # footprints: eigenvalues over five decades, random rotation, plus the dilation
    l1 = 10.0 ** rng.uniform(-1, 4, n)
    l2 = l1 * 10.0 ** rng.uniform(-4, 0, n)
    th = rng.uniform(0, np.pi, n)
    cs, sn = np.cos(th), np.sin(th)
    a = cs * cs * l1 + sn * sn * l2 + 0.3
    c = sn * sn * l1 + cs * cs * l2 + 0.3
    b = cs * sn * (l1 - l2)
    o = np.where(rng.uniform(0, 1, n) < 0.3, 1.0 / 255.0 * (1 + 10.0 ** rng.uniform(-6, -1, n)),
                 rng.uniform(1.0 / 255.0, 1.0, n))
    u = rng.uniform(0, 1, n)
    v = rng.uniform(0, 1, n)
    hx, hy = _rect_halfwidths(a, b, c, o)
    det = a * c - b * b
    worst = 0.0
    for i in range(n):
        # the pixels just outside the rect on each side, along the whole perimeter
        x0, x1 = np.ceil(u[i] - hx[i]), np.floor(u[i] + hx[i])
        y0, y1 = np.ceil(v[i] - hy[i]), np.floor(v[i] + hy[i])
        xs = np.arange(x0 - 1, x1 + 2)
        ys = np.arange(y0 - 1, y1 + 2)
        ring = np.concatenate([
            np.stack([xs, np.full_like(xs, y0 - 1)], 1), np.stack([xs, np.full_like(xs, y1 + 1)], 1),
            np.stack([np.full_like(ys, x0 - 1), ys], 1), np.stack([np.full_like(ys, x1 + 1), ys], 1)])
        if ring.shape[0] > 20000:
            ring = ring[rng.choice(ring.shape[0], 20000, replace=False)]
        dx = ring[:, 0] - u[i]
        dy = ring[:, 1] - v[i]
        sigma = 0.5 * (c[i] * dx * dx - 2.0 * b[i] * dx * dy + a[i] * dy * dy) / det[i]
        alpha = o[i] * np.exp(-sigma)
        worst = max(worst, float(alpha.max()) * 255.0)
    assert worst <= 0.9753, worst


def test_margin_check_fails_for_the_unwidened_rect():
    """The same check against a rect built at q = 2 ln(255 o) with no cap margin
    finds pixels whose alpha is within a hair of the threshold (so the
    property above is not vacuous)."""
    rng = np.random.default_rng(11)
    n = 2000
    l1 = 10.0 ** rng.uniform(-1, 3, n)
    a = l1 + 0.3
    c = l1 + 0.3
    o = rng.uniform(0.05, 1.0, n)
    q = 2.0 * np.log(255.0 * o)
    h = np.sqrt(q * a)
    u = rng.uniform(0, 1, n)
    worst = 0.0
    for i in range(n):
        x1 = np.floor(u[i] + h[i])
        dx = x1 + 1 - u[i]
        worst = max(worst, o[i] * np.exp(-0.5 * dx * dx / a[i]) * 255.0)
    assert worst > 0.99, worst
