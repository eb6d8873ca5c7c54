"""The whole step captured in a HIP graph and replayed: every replay equals
the eager result (forward bitwise; gradients within float-atomic
reordering), with eager work and synchronisation between replays, and pose
updates written in place are picked up by later replays."""
import numpy as np
import pytest
import torch

from paper_2601_00705_amd import scenes

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2601_00705_amd.render import Config, Renderer


def _step(R, P, poses, target, bufs):
    rgb, T, nc, dL, grads, d_xi = bufs
    R.project(P, poses)
    R.bin()
    R.render_fwd(rgb, T, nc)
    R.loss_l1(rgb, target, dL)
    R.raster_bwd(T, nc, dL)
    R.project_bwd(P, poses, None, grads, d_xi)


def test_graph_replays_match_eager():
    params, _ = scenes.room_scene(77, 30_000, 8_000, avoid=[np.zeros(3)])
    rng = np.random.default_rng(5)
    pose_list, _ = scenes.random_room_poses(rng, 3)
    cams = [scenes.camera(160, 120, 131.25), scenes.camera(240, 136, 120.0), scenes.camera(96, 64, 80.0)]
    cfg = Config()
    print("[graph] setup", flush=True)
    P = {k: torch.from_numpy(v).cuda() for k, v in params.items()}
    poses = torch.from_numpy(np.stack(pose_list).astype(np.float32)).cuda()
    R = Renderer(params["opacity_logit"].shape[0], cams, cfg)
    rgb0, _, _, _ = R.forward_all(P, poses)
    target = (rgb0 * 0.9 + 0.02).contiguous()
    need, _ = R.pair_count()
    R._make(int(need * 2) + 4096)
    Pt = R.total_pixels
    bufs = (torch.empty(3 * Pt, device="cuda"), torch.empty(Pt, device="cuda"),
            torch.empty(Pt, dtype=torch.int32, device="cuda"), torch.empty(3 * Pt, device="cuda"),
            {k: torch.empty_like(v) for k, v in P.items()}, torch.empty(3, 6, device="cuda"))

    def snapshot():
        rgb, T, nc, dL, grads, d_xi = bufs
        return [rgb.clone(), T.clone(), nc.clone(), d_xi.clone()] + [grads[k].clone() for k in sorted(grads)]

    _step(R, P, poses, target, bufs)
    torch.cuda.synchronize()
    eager = snapshot()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        _step(R, P, poses, target, bufs)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            _step(R, P, poses, target, bufs)
    torch.cuda.synchronize()
    print("[graph] captured", flush=True)
    for rep in range(4):
        for k in bufs[4]:
            bufs[4][k].fill_(float("nan"))
        bufs[0].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = snapshot()
        assert torch.equal(got[0], eager[0]) and torch.equal(got[1], eager[1]) and torch.equal(got[2], eager[2])
        for a, b in zip(got[3:], eager[3:]):
            scale = float(b.abs().max()) + 1e-30
            assert float((a - b).abs().max()) <= 1e-4 * scale, rep
        # eager work between replays
        _ = (target * 2).sum().item()
    # an in-place pose update is seen by the next replay
    new_pose = torch.from_numpy(scenes.left_perturb(pose_list[0], np.array([0.02, 0, 0, 0, 0.01, 0]))
                                .astype(np.float32)).cuda()
    poses[0].copy_(new_pose)
    g.replay()
    torch.cuda.synchronize()
    replayed = snapshot()
    _step(R, P, poses, target, bufs)
    torch.cuda.synchronize()
    eager2 = snapshot()
    assert torch.equal(replayed[0], eager2[0])
    assert not torch.equal(replayed[0], eager[0])
    _, ovf = R.pair_count()
    assert not ovf


def test_kernel_timing_eager_only():
    """The library's event timer brackets every launch group of an eager
    step once, with positive device time, and records nothing while the
    stream is captured into a graph."""
    from paper_2601_00705_amd import lib
    w = scenes.workload(0)
    cfg = Config()
    P = {k: torch.from_numpy(v).cuda() for k, v in w["params"].items()}
    poses = torch.from_numpy(w["poses"].astype(np.float32)).cuda()
    print("[timing] setup", flush=True)
    R = Renderer(P["opacity_logit"].shape[0], w["cams"], cfg)
    rgb0, _, _, _ = R.forward_all(P, poses)
    target = (rgb0 * 0.5).contiguous()
    Pt = R.total_pixels
    bufs = (torch.empty(3 * Pt, device="cuda"), torch.empty(Pt, device="cuda"),
            torch.empty(Pt, dtype=torch.int32, device="cuda"), torch.empty(3 * Pt, device="cuda"),
            {k: torch.empty_like(v) for k, v in P.items()}, torch.empty(1, 6, device="cuda"))
    R.set_timing(True)
    _step(R, P, poses, target, bufs)
    # the tracking-loss and mapping-loss groups, outside the L1 step
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    expo = torch.empty(1, 2, dtype=torch.float64, device="cuda")
    R.loss_track(bufs[0], bufs[1], target, 0.5, 0.05, loss, expo, torch.empty_like(bufs[0]),
                 torch.empty_like(bufs[1]))
    R.loss_mapping(bufs[0], target, 0.2, torch.empty(1, dtype=torch.float64, device="cuda"),
                   torch.empty_like(bufs[0]))
    t = R.read_timing()
    assert set(t) == set(lib.TIMERS)
    for name, (ms, cnt) in t.items():
        assert cnt == 1 and ms > 0.0, name
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            _step(R, P, poses, target, bufs)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    t2 = R.read_timing()
    assert all(t2[k][1] == 1 for k in t2), t2
    R.set_timing(False)
    assert all(v == (0.0, 0) for v in R.read_timing().values())
