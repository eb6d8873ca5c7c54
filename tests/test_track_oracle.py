"""Pins of the FP64 tracking-loss oracle (appendix, Tracking and Camera Pose
Optimization: Eqs. (app-bright), (app-ls), (app-trackloss), (app-weight)).

Each pin checks the oracle against something other than its own formulas:
a library least-squares solver, exact affine data, invariances that hold only
if (g, b) is re-fitted and differentiated through, linear ramps whose central
differences are exact, the clip's saturated regions, and central finite
differences of the loss itself.
"""
import numpy as np
import pytest

import oracle
from paper_2601_00705_amd import scenes

TA, TG = 0.6, 0.05


def _view(seed, H=9, W=11):
    cams = [dict(width=W, height=H, fx=10.0, fy=10.0, cx=W / 2, cy=H / 2)]
    rgb, T, target = scenes.track_inputs(seed, cams)
    return rgb.reshape(3, H, W).astype(np.float64), T.reshape(H, W).astype(np.float64), \
        target.reshape(3, H, W).astype(np.float64)


def test_exposure_matches_library_least_squares():
    Ih, _, I = _view(1)
    g, b, degenerate, _ = oracle.track_exposure(Ih, I)
    A = np.stack([Ih.ravel(), np.ones(Ih.size)], axis=1)
    (g_ref, b_ref), *_ = np.linalg.lstsq(A, I.ravel(), rcond=None)
    assert not degenerate
    assert abs(g - g_ref) < 1e-10 and abs(b - b_ref) < 1e-10


def test_exact_affine_observation_has_zero_loss_and_gradient():
    Ih, T, _ = _view(2)
    I = 2.0 * Ih + 0.125
    loss, (g, b), dI, dT = oracle.track_view(Ih, T, I, TA, TG)
    assert abs(g - 2.0) < 1e-12 and abs(b - 0.125) < 1e-12
    assert loss < 1e-10
    # residuals are rounding noise around 0 (their signs are arbitrary), so
    # only the transmittance gradient, which scales with |r|, must vanish
    assert np.all(np.abs(dT) < 1e-9)


def test_loss_is_invariant_to_an_affine_change_of_the_render():
    Ih, T, I = _view(3)
    l0, _, dI, _ = oracle.track_view(Ih, T, I, TA, TG)
    for a, c in ((1.7, 0.0), (1.0, -0.3), (0.4, 0.9)):
        l1, _, _, _ = oracle.track_view(a * Ih + c, T, I, TA, TG)
        assert abs(l1 - l0) <= 1e-9 * max(1.0, abs(l0))
    # so the gradient is orthogonal to the constant image and to the render
    scale = np.abs(dI).sum()
    assert abs(dI.sum()) <= 1e-9 * scale
    assert abs((dI * Ih).sum()) <= 1e-9 * scale


def test_gradient_matches_central_differences():
    Ih, T, I = _view(4)
    _, _, dI, dT = oracle.track_view(Ih, T, I, TA, TG)
    rng = np.random.default_rng(0)
    h = 1e-6
    for _ in range(24):
        c, y, x = rng.integers(0, 3), rng.integers(0, Ih.shape[1]), rng.integers(0, Ih.shape[2])
        P, M = Ih.copy(), Ih.copy()
        P[c, y, x] += h
        M[c, y, x] -= h
        fd = (oracle.track_view(P, T, I, TA, TG)[0] - oracle.track_view(M, T, I, TA, TG)[0]) / (2 * h)
        assert abs(fd - dI[c, y, x]) <= 1e-6 * max(1.0, abs(fd)), (c, y, x, fd, dI[c, y, x])
        za = (1.0 - T[y, x]) / TA
        if min(abs(za), abs(za - 1.0)) < 1e-3:
            continue  # a kink of the clip: no derivative to compare
        P, M = T.copy(), T.copy()
        P[y, x] += h
        M[y, x] -= h
        fd = (oracle.track_view(Ih, P, I, TA, TG)[0] - oracle.track_view(Ih, M, I, TA, TG)[0]) / (2 * h)
        assert abs(fd - dT[y, x]) <= 1e-6 * max(1.0, abs(fd)), (y, x, fd, dT[y, x])


def test_gradient_norm_of_linear_ramps_is_exact():
    H, W = 6, 7
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    ramp = np.stack([0.03 * xx - 0.02 * yy, 0.01 * xx + 0.04 * yy, -0.05 * xx])
    n = oracle.track_grad_norm(ramp)
    expect = np.sqrt(0.03 ** 2 + 0.02 ** 2 + 0.01 ** 2 + 0.04 ** 2 + 0.05 ** 2)
    assert np.allclose(n, expect, rtol=0, atol=1e-14)
    # an axis of extent 1 contributes nothing
    one_row = oracle.track_grad_norm(ramp[:, :1, :]) ** 2     # only x differences remain
    one_col = oracle.track_grad_norm(ramp[:, :, :1]) ** 2     # only y differences remain
    assert np.allclose(one_row, 0.03 ** 2 + 0.01 ** 2 + 0.05 ** 2, rtol=0, atol=1e-14)
    assert np.allclose(one_col, 0.02 ** 2 + 0.04 ** 2, rtol=0, atol=1e-14)
    assert np.all(oracle.track_grad_norm(ramp[:, :1, :1]) == 0.0)


def test_weights_vanish_on_flat_observation_and_empty_render():
    Ih, T, I = _view(5)
    flat = np.full_like(I, 0.4)
    loss, _, dI, dT = oracle.track_view(Ih, T, flat, TA, TG)
    assert loss == 0.0 and np.all(dT == 0.0)
    # every weight is zero, so only the (g, b) coupling could act, and it
    # multiplies sums of w s that are zero too
    assert np.all(dI == 0.0)
    loss, _, dI, dT = oracle.track_view(Ih, np.ones_like(T), I, TA, TG)  # alpha_hat = 0
    assert loss == 0.0 and np.all(dI == 0.0) and np.all(dT == 0.0)


def test_saturated_opacity_weight_has_no_transmittance_gradient():
    Ih, T, I = _view(6)
    T_sat = np.full_like(T, 0.2)  # alpha_hat = 0.8 >= tau_alpha
    _, _, _, dT = oracle.track_view(Ih, T_sat, I, TA, TG)
    assert np.all(dT == 0.0)
    # inside the ramp: dL/dT = -(1/tau_alpha) w_grad sum_c |r|
    T_in = np.full_like(T, 0.7)  # alpha_hat = 0.3 < tau_alpha
    loss, (g, b), _, dT = oracle.track_view(Ih, T_in, I, TA, TG)
    wg = np.minimum(oracle.track_grad_norm(I) / TG, 1.0)
    assert np.allclose(dT, -(1.0 / TA) * wg * np.abs(I - g * Ih - b).sum(axis=0), rtol=1e-12, atol=0)
    assert np.isclose(loss, (0.3 / TA * wg * np.abs(I - g * Ih - b).sum(axis=0)).sum(), rtol=1e-12)


def test_constant_render_takes_unit_gain():
    _, T, I = _view(7)
    Ih = np.full_like(I, 0.25)
    loss, (g, b), dI, _ = oracle.track_view(Ih, T, I, TA, TG)
    assert g == 1.0 and abs(b - (I.mean() - 0.25)) < 1e-12
    # shifting the constant render is absorbed by b
    l2, _, _, _ = oracle.track_view(Ih + 0.1, T, I, TA, TG)
    assert abs(l2 - loss) < 1e-10 * max(1.0, loss)
    assert abs(dI.sum()) < 1e-9 * max(1.0, np.abs(dI).sum())


def test_views_are_independent():
    cams = [dict(width=5, height=4, fx=1.0, fy=1.0, cx=2.0, cy=2.0),
            dict(width=3, height=6, fx=1.0, fy=1.0, cx=1.0, cy=3.0)]
    rgb, T, target = scenes.track_inputs(11, cams)
    loss, expo, d_rgb, d_T = oracle.track_loss(rgb, T, target, cams, TA, TG)
    l1, gb1, dI1, dT1 = oracle.track_view(rgb[:60].reshape(3, 4, 5), T[:20].reshape(4, 5),
                                          target[:60].reshape(3, 4, 5), TA, TG)
    assert loss[0] == l1 and tuple(expo[0]) == gb1
    assert np.array_equal(d_rgb[:60], dI1.ravel()) and np.array_equal(d_T[:20], dT1.ravel())
