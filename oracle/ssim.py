"""FP64 oracle of the mapping loss: L1 plus the structural-similarity term.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers; the product path never imports it.

The optimisation settings of the appendix combine an L1 term and an SSIM term
with weight lambda_dssim = 0.2 (Table "train_config" and the text around it):

    L = (1 - lambda) mean |I_hat - I| + lambda (1 - mean SSIM(I_hat, I))

Readings where the paper is silent:
  - SSIM is the index of Wang et al. (2004) per colour channel: an 11 x 11
    Gaussian window of standard deviation 1.5 (weights normalised to sum 1
    over the window), C1 = (0.01 L)^2, C2 = (0.03 L)^2 with dynamic range
    L = 1, and windows that reach outside the image read zeros (the image is
    zero-padded; every pixel has an SSIM value);
  - SSIM(p) = (2 mu_x mu_y + C1)(2 sigma_xy + C2)
              / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2)),
    with the local moments mu_x = w * x, sigma_x^2 = w * x^2 - mu_x^2,
    sigma_xy = w * (x y) - mu_x mu_y (w * . the window-weighted sum);
  - both means run over every pixel and channel of every view of the batch
    (as the L1 gradient seed does); the loss is one number;
  - the gradient is taken with respect to the render x; d|r|/dr at r = 0 is 0.

The local moments are windowed sums written out offset by offset (no
separable filtering); the gradient is the chain rule through them: the
adjoint of a zero-padded window sum with a symmetric window is the same
window sum.
"""
from __future__ import annotations

import numpy as np

RADIUS = 5
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window():
    """The 1-D Gaussian weights of offsets -5..5, normalised to sum 1."""
    i = np.arange(-RADIUS, RADIUS + 1, dtype=np.float64)
    w = np.exp(-(i * i) / (2.0 * SIGMA * SIGMA))
    return w / w.sum()


def window_sum(img):
    """sum over offsets (a, b) in the 11 x 11 window of w_a w_b img(p + (a, b)),
    zero outside the image; img [H][W] float64."""
    w = window()
    H, W = img.shape
    P = np.pad(np.asarray(img, np.float64), RADIUS)
    out = np.zeros((H, W))
    for a in range(2 * RADIUS + 1):
        for b in range(2 * RADIUS + 1):
            out += w[a] * w[b] * P[a:a + H, b:b + W]
    return out


def ssim_map(x, y):
    """SSIM of every pixel of one channel pair x, y [H][W]; also returns the
    partial derivatives of SSIM(p) with respect to the local moments
    mu_x(p), w * x^2 (p) and w * (x y) (p)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = window_sum(x), window_sum(y)
    mxx, myy, mxy = window_sum(x * x), window_sum(y * y), window_sum(x * y)
    vx, vy, cxy = mxx - mx * mx, myy - my * my, mxy - mx * my
    A1, A2 = 2.0 * mx * my + C1, 2.0 * cxy + C2
    B1, B2 = mx * mx + my * my + C1, vx + vy + C2
    S = A1 * A2 / (B1 * B2)
    # S = A1 A2 / (B1 B2); mu_x enters A1 (2 mu_y), A2 (-2 mu_y), B1 (2 mu_x)
    # and B2 (-2 mu_x); w * x^2 enters B2 (1); w * (x y) enters A2 (2)
    d_mx = 2.0 * my * (A2 - A1) / (B1 * B2) - 2.0 * mx * S * (1.0 / B1 - 1.0 / B2)
    d_mxx = -S / B2
    d_mxy = 2.0 * A1 / (B1 * B2)
    return S, d_mx, d_mxx, d_mxy


def ssim_grad(x, y, g):
    """d(sum_p g(p) SSIM(p))/dx for one channel."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    _, d_mx, d_mxx, d_mxy = ssim_map(x, y)
    return window_sum(g * d_mx) + 2.0 * x * window_sum(g * d_mxx) + y * window_sum(g * d_mxy)


def mapping_loss(rgbs, targets, lam):
    """rgbs, targets: lists of [3][H_v][W_v] arrays (one per view).  Returns
    (loss, [dL/d rgb_v]) in float64."""
    P = sum(r.shape[1] * r.shape[2] for r in rgbs)
    n = 3.0 * P
    l1 = 0.0
    ssum = 0.0
    grads = []
    for x, y in zip(rgbs, targets):
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        r = x - y
        l1 += np.abs(r).sum()
        g = (1.0 - lam) * np.sign(r) / n
        for c in range(3):
            S, _, _, _ = ssim_map(x[c], y[c])
            ssum += S.sum()
            g[c] -= lam / n * ssim_grad(x[c], y[c], np.ones_like(S))
        grads.append(g)
    loss = (1.0 - lam) * l1 / n + lam * (1.0 - ssum / n)
    return loss, grads
