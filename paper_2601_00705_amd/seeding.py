"""One-shot Gaussian seeding on the GPU (argument marshalling for the C ABI's
gsr_seed_triangulate, gsr_seed_scale and gsr_seed_frame; every step runs in
the library)."""
from __future__ import annotations

import torch

from . import lib

PARAM_KEYS = ("mean", "quat", "log_scale", "opacity_logit", "colour")


def _stream(device):
    return torch.cuda.current_stream(device).cuda_stream


def triangulate(views, cfg, x_ref, x_nb, kappa, diagnostics=True):
    """views: [reference, neighbours...] dicts with P (3x4), centre (3), width,
    height, image (device [3][H][W] float32), gain, bias.  x_ref [2][n],
    x_nb [K][2][n], kappa [K][n]: device float32.  Returns a dict of device
    tensors: mean [3][n], colour [3][n], opacity_logit [n], valid [n] int32
    and, with diagnostics, best, err, angle, kappa_bar."""
    n = int(x_ref.shape[-1])
    dev = x_ref.device
    out = {"mean": torch.empty(3, n, device=dev), "colour": torch.empty(3, n, device=dev),
           "opacity_logit": torch.empty(n, device=dev), "valid": torch.empty(n, dtype=torch.int32, device=dev)}
    if diagnostics:
        out.update(best=torch.empty(n, dtype=torch.int32, device=dev), err=torch.empty(n, device=dev),
                   angle=torch.empty(n, device=dev), kappa_bar=torch.empty(n, device=dev))
    lib.gsr_seed_triangulate(views, cfg, x_ref, x_nb, kappa, out["mean"], out["colour"], out["opacity_logit"],
                             out["valid"], out.get("best"), out.get("err"), out.get("angle"), out.get("kappa_bar"),
                             _stream(dev))
    return out


class Scaler:
    """Holds the workspace of gsr_seed_scale for up to n seeds."""

    def __init__(self, n, device="cuda"):
        self.n = int(n)
        self.workspace = torch.empty(max(lib.gsr_seed_scale_workspace_bytes(self.n), 1), dtype=torch.uint8,
                                     device=device)

    def __call__(self, mean, valid, floor_scale=1e-4, log_scale=None):
        n = int(mean.shape[-1])
        if n > self.n:
            raise ValueError(f"{n} seeds exceed the workspace's {self.n}")
        if log_scale is None:
            log_scale = torch.empty(3, n, device=mean.device)
        lib.gsr_seed_scale(n, mean, valid, floor_scale, self.workspace, log_scale, _stream(mean.device))
        return log_scale

    def frame(self, mean, valid, err, angle, P_ref, centre_ref, radius, c_par=1.0, floor_scale=1e-4,
              quat=None, log_scale=None):
        """Anisotropic initialisation of Eq. (app-sigma-init): (quat [4][n],
        log_scale [3][n]) of the seeds, from the plane fitted to the seeds
        within `radius` and the reference view P_ref (3x4), centre_ref."""
        n = int(mean.shape[-1])
        if n > self.n:
            raise ValueError(f"{n} seeds exceed the workspace's {self.n}")
        if quat is None:
            quat = torch.empty(4, n, device=mean.device)
        if log_scale is None:
            log_scale = torch.empty(3, n, device=mean.device)
        P = [float(x) for row in P_ref for x in row] if hasattr(P_ref[0], "__len__") else list(P_ref)
        lib.gsr_seed_frame(n, mean, valid, err, angle, P, centre_ref, radius, c_par, floor_scale, self.workspace,
                           quat, log_scale, _stream(mean.device))
        return quat, log_scale


def gaussians(seeds, log_scale, quat=None):
    """The valid seeds as Gaussian parameters in the renderer's layout
    (identity rotation unless quat [4][n] is given)."""
    keep = seeds["valid"] != 0
    m = int(keep.sum())
    if quat is None:
        quat = torch.zeros(4, m, device=seeds["mean"].device)
        quat[0] = 1.0
    else:
        quat = quat[:, keep].contiguous()
    return {"mean": seeds["mean"][:, keep].contiguous(), "quat": quat,
            "log_scale": log_scale[:, keep].contiguous(),
            "opacity_logit": seeds["opacity_logit"][keep].contiguous(),
            "colour": seeds["colour"][:, keep].contiguous()}
