"""The per-view completion stamps of the backward (the layout's stamps):
every view of a step gets a completion time after the step's start, a
second step moves them all forward, and a second backward of the same
forward stamps again."""
import numpy as np
import pytest
import torch

from paper_2601_00705_amd import scenes
from paper_2601_00705_amd.render import Config, Renderer
from helpers import to_dev

pytestmark = pytest.mark.gpu


def test_view_stamps_follow_the_steps():
    params, cam = scenes.cloud(55, 2000, 64, 48, 50.0)
    cams = [cam, dict(cam, width=40, height=30, cx=20.0, cy=15.0), dict(cam)]
    poses = np.stack([scenes.identity_pose()] * 3).astype(np.float32)
    R = Renderer(2000, cams, Config())
    P = to_dev(params)
    poses_d = torch.from_numpy(poses).cuda()
    Ptot = sum(c["width"] * c["height"] for c in cams)
    dL = torch.from_numpy(scenes.upstream_grad(1, 3 * Ptot)).cuda()
    prev = None
    for step in range(2):
        rgb, T, nc, _ = R.forward_all(P, poses_d)
        R.raster_bwd(T, nc, dL)
        torch.cuda.synchronize()
        s = R.stamps().cpu().numpy().astype(np.int64).copy()
        start, ends = s[-1], s[:-1]
        assert np.all(ends >= start), (start, ends)
        lat = R.view_latency_ms().numpy()
        assert np.all((lat >= 0) & (lat < 1e4)), lat
        if prev is not None:
            assert start >= prev.max()
        prev = s
    # a second backward of the same forward stamps again
    R.raster_bwd(T, nc, dL)
    torch.cuda.synchronize()
    s2 = R.stamps().cpu().numpy().astype(np.int64)
    assert np.all(s2[:-1] >= prev[:-1]) and s2[-1] == prev[-1]
