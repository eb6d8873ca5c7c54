"""Pins of the FP64 mapping-loss oracle (L1 + lambda (1 - SSIM)) against
what the mathematics fixes: an independent library filter for the local
moments, closed forms of SSIM for identical, constant, shifted and negated
images, the L1 special case, and central finite differences of the loss."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import ssim as M


def _gauss(img):
    # scipy's Gaussian filter with the same window: radius int(truncate*sigma + 0.5) = 5
    return ndimage.gaussian_filter(np.asarray(img, np.float64), sigma=1.5, mode="constant", cval=0.0,
                                   truncate=5.0 / 1.5)


def test_window_sum_is_the_truncated_gaussian_filter():
    rng = np.random.default_rng(0)
    for shape in [(1, 1), (3, 17), (23, 9), (40, 41)]:
        img = rng.uniform(size=shape)
        assert np.allclose(M.window_sum(img), _gauss(img), rtol=1e-13, atol=1e-15)
    assert np.isclose(M.window().sum(), 1.0) and np.allclose(M.window(), M.window()[::-1])


def test_identical_images_score_one_and_are_stationary():
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(3, 12, 19))
    for c in range(3):
        S = M.ssim_map(x[c], x[c])[0]
        assert np.allclose(S, 1.0, rtol=0, atol=1e-12)
    loss, g = M.mapping_loss([x], [x], 1.0)
    assert abs(loss) < 1e-12 and np.abs(g[0]).max() < 1e-12


def test_constant_images_closed_form():
    a, b = 0.3, 0.7
    x = np.full((30, 31), a)
    y = np.full((30, 31), b)
    S = M.ssim_map(x, y)[0]
    inner = S[5:-5, 5:-5]
    assert np.allclose(inner, (2 * a * b + M.C1) / (a * a + b * b + M.C1), rtol=1e-12)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_shifted_and_negated_images(sign):
    """y = s x + c away from the border: sigma_y^2 = sigma_x^2 and
    sigma_xy = s sigma_x^2, so SSIM = l(mu_x, mu_y) (C2 + 2 s v) / (C2 + 2 v),
    with the moments taken from scipy's filter."""
    rng = np.random.default_rng(2)
    x = rng.uniform(size=(32, 33))
    c = 0.25 if sign > 0 else 1.0
    y = sign * x + c
    S = M.ssim_map(x, y)[0][5:-5, 5:-5]
    mx = _gauss(x)[5:-5, 5:-5]
    vx = _gauss(x * x)[5:-5, 5:-5] - mx * mx
    my = sign * mx + c
    lum = (2 * mx * my + M.C1) / (mx * mx + my * my + M.C1)
    want = lum * (M.C2 + 2 * sign * vx) / (M.C2 + 2 * vx)
    assert np.allclose(S, want, rtol=1e-10, atol=1e-13)


def test_symmetric_in_the_two_images():
    rng = np.random.default_rng(3)
    x, y = rng.uniform(size=(2, 14, 15))
    assert np.allclose(M.ssim_map(x, y)[0], M.ssim_map(y, x)[0], rtol=1e-13)


def test_lambda_zero_is_the_l1_seed():
    rng = np.random.default_rng(4)
    xs = [rng.uniform(size=(3, 6, 7)), rng.uniform(size=(3, 4, 11))]
    ys = [rng.uniform(size=(3, 6, 7)), rng.uniform(size=(3, 4, 11))]
    ys[0][1, 2, 3] = xs[0][1, 2, 3]  # a zero residual takes sign 0
    loss, g = M.mapping_loss(xs, ys, 0.0)
    n = 3 * (6 * 7 + 4 * 11)
    assert np.isclose(loss, sum(np.abs(x - y).sum() for x, y in zip(xs, ys)) / n, rtol=1e-14)
    for x, y, gv in zip(xs, ys, g):
        assert np.array_equal(gv, np.sign(x - y) / n)
    assert g[0][1, 2, 3] == 0.0


def test_gradient_matches_central_differences():
    """lambda = 1 (smooth): every pixel of one channel of two views of
    different sizes, including pixels within the window radius of every
    border."""
    rng = np.random.default_rng(5)
    xs = [rng.uniform(size=(3, 7, 9)), rng.uniform(size=(3, 12, 4))]
    ys = [rng.uniform(size=(3, 7, 9)), rng.uniform(size=(3, 12, 4))]
    _, g = M.mapping_loss(xs, ys, 1.0)
    h = 1e-6
    for v in range(2):
        fd = np.zeros(xs[v].shape[1:])
        for pix in np.ndindex(*fd.shape):
            idx = (1,) + pix
            xp = [x.copy() for x in xs]
            xm = [x.copy() for x in xs]
            xp[v][idx] += h
            xm[v][idx] -= h
            fd[pix] = (M.mapping_loss(xp, ys, 1.0)[0] - M.mapping_loss(xm, ys, 1.0)[0]) / (2 * h)
        # the differences carry ~1e-10 of rounding noise (loss ~1, h = 1e-6)
        assert np.allclose(g[v][1], fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max())


def test_mixed_loss_value_and_gradient():
    """(1 - lambda) L1 + lambda D-SSIM is the weighted sum of the two parts."""
    rng = np.random.default_rng(6)
    xs = [rng.uniform(size=(3, 9, 10))]
    ys = [rng.uniform(size=(3, 9, 10))]
    l0, g0 = M.mapping_loss(xs, ys, 0.0)
    l1, g1 = M.mapping_loss(xs, ys, 1.0)
    l, g = M.mapping_loss(xs, ys, 0.2)
    assert np.isclose(l, 0.8 * l0 + 0.2 * l1, rtol=1e-14)
    assert np.allclose(g[0], 0.8 * g0[0] + 0.2 * g1[0], rtol=1e-13, atol=1e-18)
