"""Pins of the oracle's SSIM term (mapping loss, Sec. 3.4) against what the
definition and the mathematics fix, independently of the oracle's code."""
import numpy as np
import pytest

from oracle import oracle as O


def _window2d():
    # the window from a library routine, not from the oracle's formula
    from scipy.signal.windows import gaussian
    g = gaussian(2 * O.SSIM_RADIUS + 1, O.SSIM_SIGMA)
    g = g / g.sum()
    return np.outer(g, g)


def test_window_matches_library_gaussian():
    w = _window2d()
    np.testing.assert_allclose(np.outer(O.ssim_window(), O.ssim_window()), w, rtol=1e-14, atol=0)
    assert abs(O.ssim_window().sum() - 1.0) < 1e-15


def _brute_ssim(x, y):
    """Per pixel, plain loops over the 2D window; pixels outside the image
    contribute zero."""
    H, W = x.shape
    w = _window2d()
    R = O.SSIM_RADIUS
    out = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            m = [0.0] * 5
            for a in range(-R, R + 1):
                for b in range(-R, R + 1):
                    ii, jj = i + a, j + b
                    if 0 <= ii < H and 0 <= jj < W:
                        wt = w[a + R, b + R]
                        xv, yv = x[ii, jj], y[ii, jj]
                        m[0] += wt * xv
                        m[1] += wt * yv
                        m[2] += wt * xv * xv
                        m[3] += wt * yv * yv
                        m[4] += wt * xv * yv
            mx, my, exx, eyy, exy = m
            vx, vy, cxy = exx - mx * mx, eyy - my * my, exy - mx * my
            out[i, j] = ((2 * mx * my + O.SSIM_C1) * (2 * cxy + O.SSIM_C2)) / \
                        ((mx * mx + my * my + O.SSIM_C1) * (vx + vy + O.SSIM_C2))
    return out


@pytest.mark.parametrize("shape", [(7, 9), (13, 17)])
def test_ssim_matches_brute_force_windows(shape):
    rng = np.random.default_rng(11)
    x, y = rng.random(shape), rng.random(shape)
    np.testing.assert_allclose(O.ssim_channel(x, y), _brute_ssim(x, y), rtol=1e-12, atol=1e-12)


def test_identical_images_give_one_and_zero_gradient():
    rng = np.random.default_rng(3)
    x = rng.random((19, 23))
    s, g = O.ssim_channel(x, x, grad=True)
    np.testing.assert_allclose(s, 1.0, rtol=0, atol=1e-14)
    assert np.abs(g).max() < 1e-12


def test_symmetry():
    rng = np.random.default_rng(4)
    x, y = rng.random((15, 21)), rng.random((15, 21))
    np.testing.assert_allclose(O.ssim_channel(x, y), O.ssim_channel(y, x), rtol=1e-13, atol=1e-14)


def test_constant_images_closed_form():
    """Away from the border every window sees the constants, the variances
    vanish, and s = (2ab + C1) / (a^2 + b^2 + C1)."""
    a, b = 0.7, 0.2
    s = O.ssim_channel(np.full((30, 31), a), np.full((30, 31), b))
    R = O.SSIM_RADIUS
    want = (2 * a * b + O.SSIM_C1) / (a * a + b * b + O.SSIM_C1)
    np.testing.assert_allclose(s[R:-R, R:-R], want, rtol=1e-12)


def test_scaled_image_closed_form():
    """y = c x: sigma_y^2 = c^2 sigma_x^2, sigma_xy = c sigma_x^2, mu_y = c mu_x,
    so s = (2c mu^2 + C1)(2c v + C2) / (((1 + c^2) mu^2 + C1)((1 + c^2) v + C2))
    with mu and v the window mean and variance of x (computed here by brute
    force on one interior pixel)."""
    rng = np.random.default_rng(5)
    x = 0.2 + 0.5 * rng.random((25, 25))
    c = 0.6
    s = O.ssim_channel(x, c * x)
    w = _window2d()
    i = j = 12
    R = O.SSIM_RADIUS
    patch = x[i - R:i + R + 1, j - R:j + R + 1]
    mu = float((w * patch).sum())
    v = float((w * patch * patch).sum()) - mu * mu
    want = (2 * c * mu * mu + O.SSIM_C1) * (2 * c * v + O.SSIM_C2) / \
           (((1 + c * c) * mu * mu + O.SSIM_C1) * ((1 + c * c) * v + O.SSIM_C2))
    assert abs(s[i, j] - want) < 1e-12


def test_gradient_matches_torch_autograd():
    """A dense torch-FP64 SSIM (conv2d with the library window, zero padding)
    differentiated by autograd equals the oracle's hand-derived gradient."""
    import torch
    rng = np.random.default_rng(6)
    x, y = rng.random((17, 22)), rng.random((17, 22))
    w = torch.tensor(_window2d())[None, None]
    X = torch.tensor(x, requires_grad=True)
    Y = torch.tensor(y)

    def wm(t):
        return torch.nn.functional.conv2d(t[None, None], w, padding=O.SSIM_RADIUS)[0, 0]

    mx, my = wm(X), wm(Y)
    vx, vy, cxy = wm(X * X) - mx * mx, wm(Y * Y) - my * my, wm(X * Y) - mx * my
    smap = (2 * mx * my + O.SSIM_C1) * (2 * cxy + O.SSIM_C2) / ((mx * mx + my * my + O.SSIM_C1) * (vx + vy + O.SSIM_C2))
    smap.sum().backward()
    s, g = O.ssim_channel(x, y, grad=True)
    np.testing.assert_allclose(s, smap.detach().numpy(), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(g, X.grad.numpy(), rtol=1e-10, atol=1e-12)


class _Cam:
    def __init__(self, w, h):
        self.width, self.height = w, h


def test_view_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(7)
    cams = [_Cam(9, 7), _Cam(6, 8)]
    n = sum(3 * c.width * c.height for c in cams)
    img, ref = rng.random(n), rng.random(n)
    wts = [0.3, 1.7]
    S, g = O.ssim_views(cams, img, ref, wts)

    def loss(im):
        s, _ = O.ssim_views(cams, im, ref)
        return float(sum(wv * (1.0 - sv) for wv, sv in zip(wts, s)))

    h = 1e-6
    for i in rng.choice(n, 25, replace=False):
        e = np.zeros(n)
        e[i] = h
        fd = (loss(img + e) - loss(img - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])
