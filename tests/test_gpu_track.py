"""Parity of the tracking loss (gsr_loss_track through the C ABI) with the
FP64 oracle: appendix, Tracking and Camera Pose Optimization, Eqs.
(app-bright), (app-ls), (app-trackloss), (app-weight).

Bar: loss and exposure (g, b) within 1e-9 relative (both sides sum in FP64,
in different orders); the gradient seed (FP64 arithmetic stored as FP32)
within 1e-6 relative per element plus 1e-7 of the largest magnitude.  The
L1 subgradient is decided by the sign of each residual: elements whose
oracle residual lies within 1e-9 of zero are excluded and counted.  The
opacity and gradient weights are taken from the same FP32 inputs in FP64 on
both sides, so their clip decisions agree.  End to end, the loss seeds the
compositing backward and the gradients meet the renderer's bar.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2601_00705_amd import scenes
from tests.helpers import grad_violations, oracle_cfg, to_dev

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2601_00705_amd.render import Config, Renderer

TA, TG = 0.6, 0.05


def say(msg):
    print(msg, flush=True)


def _cams(sizes):
    return [scenes.camera(w, h, 0.8 * max(w, h)) for w, h in sizes]


def _gpu_track(R, rgb, T, target, ta=TA, tg=TG, with_dT=True):
    V = len(R.cams)
    loss = torch.empty(V, dtype=torch.float64, device="cuda")
    expo = torch.empty(V, 2, dtype=torch.float64, device="cuda")
    dI = torch.empty_like(rgb)
    dT = torch.empty_like(T) if with_dT else None
    R.loss_track(rgb, T, target, ta, tg, loss, expo, dI, dT)
    torch.cuda.synchronize()
    return loss, expo, dI, dT


def _residual_mask(rgb, target, expo, cams):
    """Per element: the oracle residual is clear of zero."""
    keep, off = [], 0
    for v, c in enumerate(cams):
        hw = 3 * int(c["width"]) * int(c["height"])
        g, b = expo[v]
        r = target[off:off + hw].astype(np.float64) - (g * rgb[off:off + hw].astype(np.float64) + b)
        keep.append(np.abs(r) > 1e-9)
        off += hw
    return np.concatenate(keep)


def _compare(cams, rgb, T, target, ta=TA, tg=TG):
    R = Renderer(1, cams, Config())
    d = {k: torch.from_numpy(x).cuda() for k, x in (("rgb", rgb), ("T", T), ("target", target))}
    loss, expo, dI, dT = _gpu_track(R, d["rgb"], d["T"], d["target"], ta, tg)
    ref_loss, ref_expo, ref_dI, ref_dT = oracle.track_loss(rgb, T, target, cams, ta, tg)
    loss, expo, dI, dT = (x.cpu().numpy() for x in (loss, expo, dI, dT))
    say(f"  loss {loss} vs {ref_loss}; exposure {expo.tolist()}")
    assert np.allclose(loss, ref_loss, rtol=1e-9, atol=1e-12)
    assert np.allclose(expo, ref_expo, rtol=1e-9, atol=1e-12)
    keep = _residual_mask(rgb, target, ref_expo, cams)
    say(f"  residual signs excluded: {int((~keep).sum())} of {keep.size}")
    for name, g, ref in (("dL_drgb", dI, ref_dI), ("dL_dT", dT, ref_dT)):
        m = keep if name == "dL_drgb" else np.ones(ref.shape, bool)
        tol = 1e-6 * np.abs(ref) + 1e-7 * max(np.abs(ref).max(), 1e-30)
        bad = (np.abs(g.astype(np.float64) - ref) > tol) & m
        say(f"  {name}: max |d| {np.abs(g - ref).max():.3g} (max |ref| {np.abs(ref).max():.3g}), {int(bad.sum())} over")
        assert not bad.any(), name
    return R, loss, expo


@pytest.mark.parametrize("seed", [1, 2])
def test_track_parity_uneven_views(seed):
    """Views of uneven sizes, including one-pixel-wide and 2x2 images, in one
    call; several blocks per view and ragged tails."""
    cams = _cams([(640, 480), (33, 17), (1, 9), (7, 1), (2, 2), (300, 200)])
    say(f"[track] uneven views, seed {seed}")
    rgb, T, target = scenes.track_inputs(seed, cams)
    _compare(cams, rgb, T, target)


def test_track_parity_thresholds():
    """Other weight thresholds: most pixels saturated (small tau), most on the
    ramps (large tau)."""
    cams = _cams([(96, 64), (50, 70)])
    rgb, T, target = scenes.track_inputs(9, cams)
    for ta, tg in ((0.05, 0.001), (3.0, 2.0)):
        say(f"[track] tau_alpha {ta}, tau_grad {tg}")
        _compare(cams, rgb, T, target, ta, tg)


def test_track_degenerate_and_empty_weight_cases():
    """A constant render takes g = 1; a flat observation or an empty render
    weights every pixel zero."""
    cams = _cams([(40, 30), (16, 16), (25, 9)])
    rgb, T, target = scenes.track_inputs(3, cams)
    rgb[:3 * 1200] = 0.25                        # view 0: constant render
    target[3 * 1200:3 * 1456] = 0.5              # view 1: flat observation
    T[1456:] = 1.0                               # view 2: nothing rendered
    say("[track] degenerate cases")
    R, loss, expo = _compare(cams, rgb, T, target)
    assert expo[0, 0] == 1.0
    assert loss[1] == 0.0 and loss[2] == 0.0


def test_track_deterministic_and_graph_replays():
    """Two calls agree bitwise, and so does every replay of a captured graph
    (no memset nodes: every partial slot is overwritten)."""
    cams = _cams([(320, 240), (64, 48)])
    rgb, T, target = (torch.from_numpy(x).cuda() for x in scenes.track_inputs(4, cams))
    R = Renderer(1, cams, Config())
    a = _gpu_track(R, rgb, T, target)
    b = _gpu_track(R, rgb, T, target)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    V = len(cams)
    loss = torch.empty(V, dtype=torch.float64, device="cuda")
    expo = torch.empty(V, 2, dtype=torch.float64, device="cuda")
    dI, dT = torch.empty_like(rgb), torch.empty_like(T)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        R.loss_track(rgb, T, target, TA, TG, loss, expo, dI, dT)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            R.loss_track(rgb, T, target, TA, TG, loss, expo, dI, dT)
    torch.cuda.synchronize()
    for rep in range(3):
        for x in (loss, expo, dI, dT):
            x.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for x, y in zip((loss, expo, dI, dT), a):
            assert torch.equal(x, y), rep
        _ = (target * 2).sum().item()


def test_track_seeds_backward_end_to_end():
    """Render -> tracking loss -> backward on the GPU against the oracle's
    render -> tracking loss -> backward, two views with a pose twist."""
    params, cam = scenes.cloud(211, 60, 48, 40, 40.0)
    cam2 = scenes.camera(36, 30, 32.0)
    p1 = scenes.left_perturb(scenes.identity_pose(), np.array([0.03, -0.02, 0.05, 0.04, -0.03, 0.02]))
    p2 = scenes.left_perturb(scenes.identity_pose(), np.array([-0.02, 0.01, 0.02, -0.03, 0.02, 0.01]))
    cams = [cam, cam2]
    poses = np.stack([p1, p2]).astype(np.float32)
    cfg = Config()
    _, _, target = scenes.track_inputs(21, cams)
    say("[track] end to end")
    R = Renderer(params["opacity_logit"].shape[0], cams, cfg)
    P = to_dev(params)
    poses_d = torch.from_numpy(poses).cuda()
    rgb, T, nc, _ = R.forward_all(P, poses_d)
    loss, expo, dI, dT = _gpu_track(R, rgb, T, torch.from_numpy(target).cuda())
    grads = {k: torch.empty_like(v) for k, v in P.items()}
    d_xi = torch.empty(2, 6, device="cuda")
    R.render_bwd(P, poses_d, T, nc, dI, dT, None, grads, d_xi)
    torch.cuda.synchronize()

    ref = oracle.render(params, cams, poses, oracle_cfg(cfg))
    # every pixel of this scene takes its compositing decisions the same way
    # in float32 (clear ratio above 1), so the strict bar applies throughout
    assert ref["clear"].min() > 1.0
    r_loss, r_expo, r_dI, r_dT = oracle.track_loss(ref["rgb"], ref["T_final"], target, cams, TA, TG)
    assert np.allclose(loss.cpu().numpy(), r_loss, rtol=1e-4)
    assert np.allclose(expo.cpu().numpy(), r_expo, rtol=1e-5, atol=1e-6)
    gref = oracle.backward(params, cams, poses, oracle_cfg(cfg), r_dI, r_dT)
    for k in ("mean", "quat", "log_scale", "opacity_logit", "colour", "xi"):
        g = (d_xi if k == "xi" else grads[k]).cpu().numpy()
        frac, ratio = grad_violations(g, gref[k])
        say(f"  {k}: violating={frac:.3%} worst={ratio:.3g}")
        assert np.all(np.isfinite(g))
        assert frac == 0.0, (k, frac, ratio)
