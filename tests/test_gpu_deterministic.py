"""The deterministic backward (gsr_config.deterministic = 1): the compositing
backward adds each tile's totals exactly, as fixed-point numbers with
integer atomics, so that every backward output is bitwise reproducible
whatever order the tiles run in.

Bar.  Against the oracle: the backward bar of the FP64-atomic path (the
sums are exact here, the FP64 path's are within ~1e-16).  Bitwise: two
calls, LDS batches of 64, 128 and 256 records (same per-entry totals,
different schedules), a batched plan against one plan per view (same tiles,
different global tile ids and order), and every replay of a captured graph.
Against the FP64-atomic mode: the screen-space accumulators within 1e-12 of
each field's largest magnitude.
"""
import numpy as np
import pytest
import torch

from paper_2601_00705_amd import scenes
from paper_2601_00705_amd.render import Config, Renderer
from helpers import to_dev
from test_gpu_parity import _check_backward

pytestmark = pytest.mark.gpu

DET = Config(deterministic=True)


def say(msg):
    print(msg, flush=True)


def _bwd(params, cams, poses, cfg, seed, R=None):
    n = params["opacity_logit"].shape[0]
    R = R or Renderer(n, cams, cfg)
    P = to_dev(params)
    poses_d = torch.from_numpy(np.ascontiguousarray(poses, dtype=np.float32)).cuda()
    rgb, T, nc, _ = R.forward_all(P, poses_d)
    Ptot = sum(c["width"] * c["height"] for c in cams)
    dL = torch.from_numpy(scenes.upstream_grad(seed, 3 * Ptot)).cuda()
    dT = torch.from_numpy(scenes.upstream_grad(seed + 1, Ptot)).cuda()
    grads = {k: torch.empty_like(v) for k, v in P.items()}
    d_xi = torch.empty(len(cams), 6, device="cuda")
    R.render_bwd(P, poses_d, T, nc, dL, dT, None, grads, d_xi)
    torch.cuda.synchronize()
    g2d = _live_grad2d(R)
    return g2d, {k: v.cpu().numpy() for k, v in grads.items()}, d_xi.cpu().numpy(), R


def _live_grad2d(R):
    """The accumulators of the projected slots, zero elsewhere (a slot the
    projection culls is never read, and its accumulators are not cleared)."""
    rec = R.records()
    live = (rec["geom"][:, 2] >= 0).cpu().numpy()
    g = rec["grad2d"].cpu().numpy().copy()
    g[~live] = 0.0
    return g


def _same(a, b):
    ga, pa, xa = a[:3]
    gb, pb, xb = b[:3]
    assert np.array_equal(ga, gb)
    for k in pa:
        assert np.array_equal(pa[k], pb[k]), k
    assert np.array_equal(xa, xb)


def test_deterministic_backward_parity_cloud_2k():
    w = scenes.workload(0)
    _check_backward("cloud-2k deterministic", w["params"], w["cams"], w["poses"], DET, 5)


def test_deterministic_backward_parity_sh3_two_views():
    params, cam = scenes.cloud(401, 80, 48, 40, 40.0, sh_degree=3)
    cams = [cam, dict(cam)]
    poses = np.stack([scenes.identity_pose(),
                      scenes.left_perturb(scenes.identity_pose(), np.array([0.05, 0.0, 0.0, 0.0, 0.03, 0.0]))])
    _check_backward("sh3 deterministic", params, cams, poses, Config(sh_degree=3, deterministic=True), 9)


def _room(seed=31):
    w = scenes.workload(1, seed=seed)
    return w["params"], w["cams"], w["poses"]


def test_bitwise_across_calls_and_batches():
    params, cams, poses = _room()
    say(f"[det] room {params['opacity_logit'].shape[0]} Gaussians")
    ref = _bwd(params, cams, poses, DET, 3)
    again = _bwd(params, cams, poses, DET, 3, R=ref[3])
    _same(ref, again)
    for batch in (64, 256):
        _same(ref, _bwd(params, cams, poses, Config(batch=batch, deterministic=True), 3))
    # the FP64-atomic mode agrees to rounding
    fp = _bwd(params, cams, poses, Config(), 3)
    scale = np.abs(ref[0]).max(axis=0) + 1e-300
    err = (np.abs(fp[0] - ref[0]) / scale).max()
    say(f"  accumulators: FP64 atomics vs fixed point, worst {err:.2e} of the field's largest")
    assert err < 1e-12


def test_bitwise_batched_against_per_view_plans():
    """Three views of different sizes in one plan, and each view in a plan of
    its own: the per-slot accumulators agree bit for bit."""
    params, cam = scenes.cloud(77, 3000, 96, 64, 60.0)
    cams = [cam, dict(cam, width=64, height=80, cx=32.0, cy=40.0), dict(cam, width=33, height=17, cx=16.5, cy=8.5)]
    poses = np.stack([scenes.identity_pose(),
                      scenes.left_perturb(scenes.identity_pose(), np.array([0.02, 0.01, 0.0, 0.01, 0.02, 0.0])),
                      scenes.left_perturb(scenes.identity_pose(), np.array([-0.03, 0.0, 0.02, 0.0, -0.01, 0.03]))])
    n = params["opacity_logit"].shape[0]
    R = Renderer(n, cams, DET)
    P = to_dev(params)
    poses_d = torch.from_numpy(poses.astype(np.float32)).cuda()
    rgb, T, nc, _ = R.forward_all(P, poses_d)
    Ptot = sum(c["width"] * c["height"] for c in cams)
    dL = torch.from_numpy(scenes.upstream_grad(4, 3 * Ptot)).cuda()
    R.raster_bwd(T, nc, dL)
    torch.cuda.synchronize()
    g_all = _live_grad2d(R)
    o3 = o1 = 0
    for v, c in enumerate(cams):
        hw = c["width"] * c["height"]
        Rv = Renderer(n, [c], DET)
        _, Tv, ncv, _ = Rv.forward_all(P, poses_d[v:v + 1])
        Rv.raster_bwd(Tv, ncv, dL[o3:o3 + 3 * hw].contiguous())
        torch.cuda.synchronize()
        assert torch.equal(Tv, T[o1:o1 + hw])
        gv = _live_grad2d(Rv)
        assert np.array_equal(gv, g_all[v * n:(v + 1) * n]), v
        o3 += 3 * hw
        o1 += hw
    say(f"  live slots with gradients: {(np.abs(g_all).sum(axis=1) > 0).sum()}")


def test_graph_replays_bitwise():
    params, cams, poses = _room(32)
    ref = _bwd(params, cams, poses, DET, 6)
    R = ref[3]
    P = to_dev(params)
    poses_d = torch.from_numpy(np.ascontiguousarray(poses, dtype=np.float32)).cuda()
    rgb, T, nc, _ = R.forward_all(P, poses_d)
    Ptot = sum(c["width"] * c["height"] for c in cams)
    dL = torch.from_numpy(scenes.upstream_grad(6, 3 * Ptot)).cuda()
    dT = torch.from_numpy(scenes.upstream_grad(7, Ptot)).cuda()
    grads = {k: torch.empty_like(v) for k, v in P.items()}
    d_xi = torch.empty(len(cams), 6, device="cuda")
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        R.render_bwd(P, poses_d, T, nc, dL, dT, None, grads, d_xi)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            R.render_bwd(P, poses_d, T, nc, dL, dT, None, grads, d_xi)
    torch.cuda.synchronize()
    for _ in range(3):
        for v in grads.values():
            v.fill_(np.nan)
        g.replay()
        torch.cuda.synchronize()
        for k in grads:
            assert np.array_equal(grads[k].cpu().numpy(), ref[1][k]), k
        assert np.array_equal(d_xi.cpu().numpy(), ref[2])
