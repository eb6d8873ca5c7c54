"""Shared test helpers: tolerances and conversions (no renderer arithmetic)."""
import numpy as np

import oracle

# Image tolerance (absolute) and gradient tolerance (per element:
# |g - g_ref| <= REL * |g_ref| + FLOOR * max |g_ref|).
IMG_ATOL = 1e-4
GRAD_REL = 1e-3
GRAD_FLOOR = 1e-5
# A pixel is "clear" when each of its compositing decisions (alpha_min skip,
# alpha_max clamp, T_min stop) lies farther from its threshold, in the FP64
# oracle, than a bound on the float32 error of the quantity compared (the
# oracle's "clear" ratio > 1; the bound follows the float32 operation count of
# the tile-centred exp2-space expansion and of the transmittance product).
# Clear pixels must match at the strict bar; the others may take a decision
# the other way, and are excluded and counted.
CLEAR = 1.0


def oracle_cfg(cfg):
    return oracle.Config(tile_w=cfg.tile_w, tile_h=cfg.tile_h, sh_degree=cfg.sh_degree, z_near=cfg.z_near,
                         dilation=cfg.dilation, alpha_min=cfg.alpha_min, alpha_max=cfg.alpha_max,
                         T_min=cfg.T_min, bg=cfg.bg, staging_f32=getattr(cfg, "precision", "fp32") == "mixed")


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


def pixel_mask(clear, cams, channels=1):
    """Boolean mask (per pixel, repeated per channel block) of the pixels
    whose decisions float32 cannot take differently (oracle clear ratio > 1)."""
    ok = clear > CLEAR
    if channels == 1:
        return ok
    parts, off = [], 0
    for c in cams:
        hw = int(c["width"]) * int(c["height"])
        parts.append(np.tile(ok[off:off + hw], channels))
        off += hw
    return np.concatenate(parts)


# Cancellation factor below which a gradient must meet the bar.  A per-pixel
# float32 addend of the backward carries the relative error of alpha (about
# 1e-6 from the tile-centred expansion) plus that of the transmittance, which
# the backward recovers by division from T_final, entry by entry from the end
# of the list: each step adds three roundings and alpha / (1 - alpha) times
# alpha's error, about 3e-7 per entry at the workloads' mean alpha of 0.1,
# so about 2e-4 at the depth of 650 entries the workloads' lists reach.  A
# sum whose addends cancel by a factor kappa (sum of magnitudes / magnitude
# of the sum) then carries up to 2e-4 kappa relative error, which can exceed
# the 1e-3 bar only when kappa >= 1e-3 / 2e-4 = 5.
KAPPA_MIN = 5.0


def cancellation(grad2d, grad2d_abs):
    """Per Gaussian: the largest cancellation factor of its screen-space
    gradients (fields u, v, A, B, C, o over every view): the sum of the
    magnitudes of the elementary products behind a field (those inside
    dL/dalpha included) over the magnitude of the field, from the oracle
    ([V][n][9] each)."""
    s = np.abs(np.asarray(grad2d)[..., :6])
    a = np.asarray(grad2d_abs)[..., :6]
    kap = np.where(a > 0, a / np.maximum(s, 1e-300), 1.0)
    return kap.max(axis=(0, 2))


def check_grad(name, g, ref, kappa=None, frac_cap=0.0, ratio_cap=1.0, say=print):
    """Every element within the bar, except (when kappa is given) elements of
    cancellation-limited Gaussians (kappa >= KAPPA_MIN): at most frac_cap of
    the elements, none beyond ratio_cap times the bar.  Returns
    (violating fraction, worst ratio)."""
    g = np.asarray(g, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert np.all(np.isfinite(g)), name
    tol = GRAD_REL * np.abs(ref) + GRAD_FLOOR * max(np.max(np.abs(ref)) if ref.size else 0.0, 1e-30)
    ratio = np.abs(g - ref) / tol
    bad = ratio > 1.0
    frac = float(bad.mean()) if ratio.size else 0.0
    worst = float(ratio.max()) if ratio.size else 0.0
    if not bad.any():
        say(f"  {name}: every element within the bar (worst {worst:.3g})")
        return frac, worst
    idx = np.nonzero(bad.reshape(-1, bad.shape[-1]).any(axis=0))[0] if bad.ndim > 1 else np.nonzero(bad)[0]
    kap = None if kappa is None else kappa[idx]
    say(f"  {name}: {int(bad.sum())} elements ({frac:.5%}) beyond the bar, worst {worst:.3g}; "
        f"their Gaussians' cancellation factors {None if kap is None else np.sort(kap)[:8]}")
    assert kappa is not None, f"{name}: {int(bad.sum())} elements beyond the bar"
    assert np.all(kap >= KAPPA_MIN), f"{name}: a Gaussian without cancellation misses the bar"
    assert frac <= frac_cap and worst <= ratio_cap, (name, frac, worst)
    return frac, worst
