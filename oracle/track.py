"""FP64 oracle of the tracking loss and its gradient seed.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers; the product path never imports it.

Follows the appendix section "Tracking and Camera Pose Optimization":
Eq. (app-bright), the affine brightness model g_I * I_hat + b_I of the
rendered image I_hat; Eq. (app-ls), (g_I, b_I) as the least-squares fit of the
observation I by that model over the image domain; Eq. (app-trackloss), the
per-pixel weighted L1 distance between I and the corrected render; and
Eq. (app-weight) with the clip definitions of w_alpha (accumulated opacity
over tau_alpha) and w_grad (observed image-gradient norm over tau_grad).

Readings where the paper is silent or loose:
  - one (g_I, b_I) per view; the least-squares problem and the L1 norm run
    over all pixels and all three colour channels of the view;
  - (g_I, b_I) is the least-squares solution as a function of the render and
    the gradient includes that dependence: substituting the solution is what
    makes the loss invariant to an affine change of the render, which is the
    stated purpose (pose updates unaffected by slow exposure drift);
  - a render without variance (N sum I_hat^2 - (sum I_hat)^2 at most 1e-12 of
    N sum I_hat^2, or all zero) takes g_I = 1 and b_I = mean(I) - mean(I_hat);
  - the accumulated opacity is alpha_hat = 1 - T_final;
  - ||grad I||_2 is the Frobenius norm, over the three channels, of the
    observation's central differences (I(x+1) - I(x-1)) / 2; one-sided
    differences at the image border; zero along an axis of extent 1;
  - d|r|/dr at r = 0 is 0, and the derivative of clip(z, 0, 1) is 1 for
    0 < z < 1 and 0 elsewhere;
  - the loss of a view is the sum over its pixels (Eq. (app-trackloss) sums
    over Omega_I), and the gradient is that of the sum over views.
"""
from __future__ import annotations

import numpy as np

# a render whose variance is below this fraction of N sum I_hat^2 counts as
# constant (exposure gain fixed at 1)
DEGENERATE_REL = 1e-12


def grad_norm(img):
    """||grad I||_2 per pixel of one observed image img[3][H][W] (float64)."""
    img = np.asarray(img, np.float64)

    def diff(axis):
        n = img.shape[axis]
        out = np.zeros_like(img)
        if n == 1:
            return out

        def sl(a, b):
            return tuple(slice(a, b) if ax == axis else slice(None) for ax in range(3))

        out[sl(1, n - 1)] = (img[sl(2, n)] - img[sl(0, n - 2)]) / 2.0
        out[sl(0, 1)] = img[sl(1, 2)] - img[sl(0, 1)]
        out[sl(n - 1, n)] = img[sl(n - 1, n)] - img[sl(n - 2, n - 1)]
        return out

    gx, gy = diff(2), diff(1)
    return np.sqrt((gx * gx + gy * gy).sum(axis=0))


def clip01(z):
    return np.minimum(np.maximum(z, 0.0), 1.0)


def exposure(I_hat, I):
    """(g, b, degenerate, sums) of Eq. (app-ls) for one view."""
    x = np.asarray(I_hat, np.float64).ravel()
    y = np.asarray(I, np.float64).ravel()
    N = float(x.size)
    Sx, Sy, Sxx, Sxy = x.sum(), y.sum(), (x * x).sum(), (x * y).sum()
    D = N * Sxx - Sx * Sx
    if not D > DEGENERATE_REL * N * Sxx:
        return 1.0, (Sy - Sx) / N, True, (N, Sx, Sy, Sxx, Sxy, D)
    g = (N * Sxy - Sx * Sy) / D
    b = (Sy - g * Sx) / N
    return g, b, False, (N, Sx, Sy, Sxx, Sxy, D)


def track_view(I_hat, T_final, I, tau_alpha, tau_grad):
    """Loss, (g, b), dL/dI_hat [3][H][W] and dL/dT_final [H][W] of one view."""
    I_hat = np.asarray(I_hat, np.float64)
    I = np.asarray(I, np.float64)
    T_final = np.asarray(T_final, np.float64)
    g, b, degenerate, (N, Sx, Sy, Sxx, Sxy, D) = exposure(I_hat, I)

    # Eq. (app-weight): w = w_alpha * w_grad
    alpha_hat = 1.0 - T_final
    za = alpha_hat / tau_alpha
    w_alpha = clip01(za)
    w_grad = clip01(grad_norm(I) / tau_grad)
    w = w_alpha * w_grad

    # Eq. (app-trackloss) with Eq. (app-bright)
    r = I - (g * I_hat + b)
    absr = np.abs(r)
    loss = float((w[None] * absr).sum())

    # gradient: explicit term, then the dependence of (g, b) on the render
    s = np.sign(r)
    dI_hat = -w[None] * s * g
    Q0 = float((w[None] * s).sum())            # -dL/db
    Q1 = float((w[None] * s * I_hat).sum())    # -dL/dg
    if degenerate:
        # b = mean(I) - mean(I_hat): db/dI_hat = -1/N, g fixed
        dI_hat = dI_hat + Q0 / N
    else:
        dg = (N * I - Sy - 2.0 * g * (N * I_hat - Sx)) / D
        db = -(Sx * dg + g) / N
        dI_hat = dI_hat - Q1 * dg - Q0 * db

    # w_alpha depends on T_final through alpha_hat = 1 - T_final
    dw_alpha = np.where((za > 0.0) & (za < 1.0), 1.0 / tau_alpha, 0.0)
    dT = -dw_alpha * w_grad * absr.sum(axis=0)
    return loss, (g, b), dI_hat, dT


def track_loss(rgb, T_final, target, cams, tau_alpha, tau_grad):
    """All views of concatenated images (the renderer's layout): rgb and
    target [sum 3 H W], T_final [sum H W].  Returns loss [V], exposure [V][2],
    dL_drgb (like rgb), dL_dT (like T_final), all float64."""
    rgb = np.asarray(rgb, np.float64).ravel()
    target = np.asarray(target, np.float64).ravel()
    T_final = np.asarray(T_final, np.float64).ravel()
    loss = np.zeros(len(cams))
    expo = np.zeros((len(cams), 2))
    d_rgb = np.zeros_like(rgb)
    d_T = np.zeros_like(T_final)
    p = 0
    for v, c in enumerate(cams):
        H, W = int(c["height"]), int(c["width"])
        hw = H * W
        l, gb, dI, dT = track_view(rgb[3 * p:3 * (p + hw)].reshape(3, H, W), T_final[p:p + hw].reshape(H, W),
                                   target[3 * p:3 * (p + hw)].reshape(3, H, W), tau_alpha, tau_grad)
        loss[v] = l
        expo[v] = gb
        d_rgb[3 * p:3 * (p + hw)] = dI.ravel()
        d_T[p:p + hw] = dT.ravel()
        p += hw
    return loss, expo, d_rgb, d_T
