"""Map maintenance on the GPU: the optimiser step with the anchor of
Eq. (app-ema), the co-visibility score of Eq. (iou), pruning and merging
with compaction, and the map's spatial storage order (the C ABI's
gsr_adam_step, gsr_covis, gsr_prune, gsr_compact, gsr_nearest, gsr_merge,
gsr_keep_list, gsr_spatial_order).
Argument marshalling only; every step runs in the library's kernels."""
from __future__ import annotations

import torch

from . import lib
from .render import _stream

PLANES = lib.PLANES
ROWS = {"mean": 3, "quat": 4, "log_scale": 3, "opacity_logit": 1}
# the appendix's optimisation settings
PAPER_LR = {"mean": 1e-3, "quat": 1e-3, "log_scale": 1e-3, "opacity_logit": 2e-3, "colour": 2e-3}


class Adam:
    """Adam state (m, v) for a Gaussian set in the renderer's plane layout,
    plus the EMA anchor of the means."""

    def __init__(self, params, lr=None, betas=(0.9, 0.999), eps=1e-8, max_grad_norm=1.0, ema=0.0,
                 anchor=True):
        self.n = int(params["opacity_logit"].shape[0])
        self.colour_rows = int(params["colour"].numel() // max(self.n, 1))
        self.lr = dict(PAPER_LR if lr is None else lr)
        self.betas, self.eps, self.max_grad_norm, self.ema = betas, eps, max_grad_norm, ema
        self.m = {k: torch.zeros_like(params[k]) for k in PLANES}
        self.v = {k: torch.zeros_like(params[k]) for k in PLANES}
        self.anchor = params["mean"].clone() if anchor else None
        dev = params["mean"].device
        self.workspace = torch.empty(lib.ADAM_WORKSPACE_BYTES, dtype=torch.uint8, device=dev)
        self.norm = torch.zeros(1, dtype=torch.float64, device=dev)
        self.t = 0

    def step(self, params, grads, lr_scale=1.0):
        """One step in place; lr_scale multiplies every rate (a schedule)."""
        self.t += 1
        cfg = lib.AdamConfig()
        for i, k in enumerate(PLANES):
            cfg.lr[i] = self.lr[k] * lr_scale
        cfg.beta1, cfg.beta2 = self.betas
        cfg.eps, cfg.max_grad_norm, cfg.ema, cfg.step = self.eps, self.max_grad_norm, self.ema, self.t
        lib.gsr_adam_step(self.n, self.colour_rows, params, grads, self.m, self.v, self.anchor, cfg,
                          self.workspace, self.norm, _stream(params["mean"].device))


def covis(T_key, T_frames, tau):
    """IoU of the visible sets of a key frame T_key [P] and frames T_frames
    [F][P] (T_final images); returns (counts [F][2] int64, iou [F] float64)."""
    F = T_frames.shape[0] if T_frames.dim() > 1 else 1
    P = T_key.numel()
    counts = torch.empty(F, 2, dtype=torch.int64, device=T_key.device)
    iou = torch.empty(F, dtype=torch.float64, device=T_key.device)
    lib.gsr_covis(P, F, T_key, T_frames, tau, counts, iou, _stream(T_key.device))
    return counts, iou


def prune(m_obs, v_vis, log_scale, opacity_logit, m_min, v_min, sigma_max, alpha_min):
    """Kept indices (in order, first `kept` entries) and kept [1] (device)."""
    n = int(opacity_logit.shape[0])
    dev = opacity_logit.device
    cfg = lib.PruneConfig(int(m_min), float(v_min), float(sigma_max), float(alpha_min))
    ws = torch.empty(max(lib.gsr_prune_workspace_bytes(n), 4), dtype=torch.uint8, device=dev)
    keep = torch.empty(n, dtype=torch.int32, device=dev)
    kept = torch.empty(1, dtype=torch.int64, device=dev)
    lib.gsr_prune(n, m_obs, v_vis, log_scale, opacity_logit, cfg, keep, kept, ws, _stream(dev))
    return keep, kept


def compact(src, keep, kept):
    """src [rows][n] or [n] -> a new tensor of the same shape whose first
    kept columns are the kept ones (the rest undefined)."""
    n = int(keep.shape[0])
    rows = src.numel() // n
    dst = torch.empty_like(src)
    lib.gsr_compact(n, rows, src, keep, kept, dst, _stream(src.device))
    return dst


def nearest(mean, valid=None):
    """Index of each Gaussian's nearest other one (-1 where none); mean
    [3][n] device, valid [n] int32 (all valid by default)."""
    n = int(mean.shape[1])
    dev = mean.device
    if valid is None:
        valid = torch.ones(n, dtype=torch.int32, device=dev)
    ws = torch.empty(max(lib.gsr_seed_scale_workspace_bytes(n), 8), dtype=torch.uint8, device=dev)
    nn = torch.empty(n, dtype=torch.int32, device=dev)
    lib.gsr_nearest(n, mean, valid, ws, nn, _stream(dev))
    return nn


def merge(params, v_vis, radius, colour_tol, nn=None):
    """Merging of mutual nearest neighbours with overlapping footprints and
    similar colours.  Returns (merged planes, keep mask [n] int32, nn):
    columns with keep 0 were merged into their partner."""
    n = int(params["opacity_logit"].shape[0])
    colour_rows = int(params["colour"].numel() // max(n, 1))
    dev = params["mean"].device
    if nn is None:
        nn = nearest(params["mean"])
    out = {k: torch.empty_like(params[k]) for k in PLANES}
    keep = torch.empty(n, dtype=torch.int32, device=dev)
    lib.gsr_merge(n, colour_rows, params, v_vis, nn, radius, colour_tol, out, keep, _stream(dev))
    return out, keep, nn


def keep_list(mask):
    """Ordered indices of the set entries of an int32 mask, and their count
    [1] (device)."""
    n = int(mask.shape[0])
    dev = mask.device
    ws = torch.empty(max(lib.gsr_prune_workspace_bytes(n), 4), dtype=torch.uint8, device=dev)
    keep = torch.empty(n, dtype=torch.int32, device=dev)
    kept = torch.empty(1, dtype=torch.int64, device=dev)
    lib.gsr_keep_list(n, mask, keep, kept, ws, _stream(dev))
    return keep, kept


# Gaussians per brick of the spatial order (see spatial_order): one
# projection wave's worth
SPATIAL_BRICK = 64


def spatial_order(mean, brick=SPATIAL_BRICK):
    """Storage order of a map whose means are [3][n] (device): index [n]
    int32, the Gaussian to store at each position.  Bricks of `brick`
    consecutive positions hold neighbours along a Morton curve over the
    map's box; consecutive bricks come from far apart."""
    n = int(mean.shape[1])
    dev = mean.device
    ws = torch.empty(max(lib.gsr_spatial_order_workspace_bytes(n), 256), dtype=torch.uint8, device=dev)
    index = torch.empty(n, dtype=torch.int32, device=dev)
    lib.gsr_spatial_order(n, mean.contiguous(), brick, index, ws, _stream(dev))
    return index


def permute(planes, index):
    """Every plane [rows][n] or [n] of `planes` (a dict of device float32
    tensors: the map, or its optimiser state) gathered by index: column j of
    the result is column index[j] of the input."""
    n = int(index.shape[0])
    kept = torch.full((1,), n, dtype=torch.int64, device=index.device)
    return {k: compact(v.contiguous(), index, kept) for k, v in planes.items()}
