"""Invariants of the GPU renderer that hold whatever the inputs: permuting
the Gaussians (distinct depths) leaves the image bit for bit and permutes
the gradients (bit for bit in the deterministic mode); a rigid motion of the
scene and the camera together leaves the image; with unit colours and a
unit background the compositing weights and T_final sum to one (Eq. (alpha));
T_final lies in [0, 1] and never grows when Gaussians are added."""
import numpy as np
import pytest
import torch

from paper_2601_00705_amd import scenes
from paper_2601_00705_amd.render import Config, Renderer
from helpers import to_dev

pytestmark = pytest.mark.gpu


def _render(params, cams, poses, cfg, dL=None):
    n = params["opacity_logit"].shape[0]
    R = Renderer(n, cams, cfg)
    P = to_dev(params)
    poses_d = torch.from_numpy(np.ascontiguousarray(poses, dtype=np.float32)).cuda()
    rgb, T, nc, _ = R.forward_all(P, poses_d)
    grads = None
    if dL is not None:
        grads = {k: torch.empty_like(v) for k, v in P.items()}
        R.render_bwd(P, poses_d, T, nc, torch.from_numpy(dL).cuda(), None, None, grads,
                     torch.empty(len(cams), 6, device="cuda"))
    torch.cuda.synchronize()
    return rgb.cpu().numpy(), T.cpu().numpy(), None if grads is None else {k: v.cpu().numpy() for k, v in grads.items()}


def test_permutation_of_the_gaussians():
    params, cam = scenes.cloud(91, 3000, 80, 60, 60.0)
    assert np.unique(params["mean"][2]).size == 3000  # distinct depths
    perm = np.random.default_rng(1).permutation(3000)
    pp = {k: np.ascontiguousarray(v[..., perm]) for k, v in params.items()}
    poses = scenes.identity_pose()[None]
    dL = scenes.upstream_grad(3, 3 * 80 * 60)
    cfg = Config(deterministic=True)
    rgb0, T0, g0 = _render(params, [cam], poses, cfg, dL)
    rgb1, T1, g1 = _render(pp, [cam], poses, cfg, dL)
    assert np.array_equal(rgb0, rgb1) and np.array_equal(T0, T1)
    for k in g0:
        assert np.array_equal(g0[k][..., perm], g1[k]), k


def _quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_rigid_motion_of_scene_and_camera():
    """x -> Q x + s for the means, q -> q_Q q for the rotations, and the
    world-to-camera pose [R | t] -> [R Q^T | t - R Q^T s]: the same image."""
    params, cam = scenes.cloud(92, 2000, 64, 48, 50.0)
    rng = np.random.default_rng(2)
    qQ = rng.normal(size=4)
    qQ /= np.linalg.norm(qQ)
    w, x, y, z = qQ
    Q = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    s = np.array([0.3, -0.2, 0.5])
    moved = dict(params)
    moved["mean"] = (Q @ params["mean"].astype(np.float64) + s[:, None]).astype(np.float32)
    moved["quat"] = np.stack([_quat_mul(qQ, q) for q in params["quat"].astype(np.float64).T], 1).astype(np.float32)
    pose = scenes.left_perturb(scenes.identity_pose(), np.array([0.02, -0.01, 0.03, 0.02, 0.01, -0.02]))
    R0, t0 = pose[:9].reshape(3, 3), pose[9:]
    R1 = R0 @ Q.T
    t1 = t0 - R1 @ s
    pose1 = np.concatenate([R1.reshape(9), t1])
    rgb0, T0, _ = _render(params, [cam], pose[None], Config())
    rgb1, T1, _ = _render(moved, [cam], pose1[None], Config())
    # the moved scene's float32 inputs differ from the original's by
    # rounding, which moves the image by much less than the 1e-4 bar
    assert np.abs(rgb0 - rgb1).max() < 1e-4 and np.abs(T0 - T1).max() < 1e-4


def test_weights_and_transmittance_sum_to_one():
    params, cam = scenes.cloud(93, 3000, 64, 48, 50.0)
    params["colour"] = np.ones_like(params["colour"])
    rgb, T, _ = _render(params, [cam], scenes.identity_pose()[None], Config(bg=(1.0, 1.0, 1.0)))
    assert np.abs(rgb - 1.0).max() < 1e-5
    assert T.min() >= 0.0 and T.max() <= 1.0 and T.min() < 0.5


def test_transmittance_never_grows_with_more_gaussians():
    params, cam = scenes.cloud(94, 3000, 64, 48, 50.0)
    half = {k: np.ascontiguousarray(v[..., :1500]) for k, v in params.items()}
    cfg = Config(T_min=0.0)
    _, T_all, _ = _render(params, [cam], scenes.identity_pose()[None], cfg)
    _, T_half, _ = _render(half, [cam], scenes.identity_pose()[None], cfg)
    assert np.all(T_all <= T_half + 1e-6)
