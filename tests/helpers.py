"""Shared test helpers: tolerances and conversions (no renderer arithmetic)."""
import numpy as np

import oracle

# Image tolerance (absolute) and gradient tolerance (per element:
# |g - g_ref| <= REL * |g_ref| + FLOOR * max |g_ref|).
IMG_ATOL = 1e-4
GRAD_REL = 1e-3
GRAD_FLOOR = 1e-5
# Pixels whose compositing decisions (alpha_min skip, alpha_max clamp, T_min
# stop) lie within this relative distance of their threshold in the FP64
# oracle may legitimately decide differently in FP32; they are excluded from
# the strict comparisons and counted.
MARGIN = 1e-3


def oracle_cfg(cfg):
    return oracle.Config(tile_w=cfg.tile_w, tile_h=cfg.tile_h, sh_degree=cfg.sh_degree, z_near=cfg.z_near,
                         dilation=cfg.dilation, alpha_min=cfg.alpha_min, alpha_max=cfg.alpha_max,
                         T_min=cfg.T_min, bg=cfg.bg)


def to_dev(params, device="cuda"):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(device) for k, v in params.items()}


def grad_violations(g, ref, rel=GRAD_REL, floor=GRAD_FLOOR):
    """Returns (fraction violating, worst ratio) of the per-element rule."""
    g = np.asarray(g, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    if ref.size == 0:
        return 0.0, 0.0
    tol = rel * np.abs(ref) + floor * max(np.max(np.abs(ref)), 1e-30)
    err = np.abs(g - ref)
    ratio = err / tol
    return float(np.mean(ratio > 1.0)), float(np.max(ratio))


def pixel_mask(margin, cams, channels=1):
    """Boolean mask (per pixel, repeated per channel block) of pixels whose
    decision margin is safe."""
    ok = margin >= MARGIN
    if channels == 1:
        return ok
    parts, off = [], 0
    for c in cams:
        hw = int(c["width"]) * int(c["height"])
        parts.append(np.tile(ok[off:off + hw], channels))
        off += hw
    return np.concatenate(parts)
