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


# The per-addend relative error that bound (2e-4, above) also gives each
# exempt element its allowance: a sum of addends of total magnitude
# kappa |g_ref| erring by up to 2e-4 of each errs by up to 2e-4 kappa |g_ref|.
EPS_TERM = 2e-4


def check_grad(name, g, ref, kappa=None, frac_cap=0.0, eps_term=EPS_TERM, kappa_min=None, say=print, rel=GRAD_REL,
               floor=GRAD_FLOOR):
    """Every element within the bar (rel |g_ref| + floor max |g_ref|),
    except, when kappa is given, elements of cancellation-limited Gaussians
    (kappa >= kappa_min, KAPPA_MIN by default): at most frac_cap of the
    elements, each within the bar plus eps_term kappa |g_ref|.  Returns
    (fraction beyond the bar, worst ratio to the bar)."""
    kappa_min = KAPPA_MIN if kappa_min is None else kappa_min
    g = np.asarray(g, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert np.all(np.isfinite(g)), name
    tol = rel * np.abs(ref) + floor * max(np.max(np.abs(ref)) if ref.size else 0.0, 1e-30)
    err = np.abs(g - ref)
    ratio = err / tol
    bad = ratio > 1.0
    frac = float(bad.mean()) if ratio.size else 0.0
    worst = float(ratio.max()) if ratio.size else 0.0
    if not bad.any():
        say(f"  {name}: every element within the bar (worst {worst:.3g})")
        return frac, worst
    assert kappa is not None, f"{name}: {int(bad.sum())} elements beyond the bar (worst {worst:.3g})"
    gauss = np.broadcast_to(np.arange(g.shape[-1]), g.shape)[bad]
    kap = np.asarray(kappa)[gauss]
    allow = tol[bad] + eps_term * kap * np.abs(ref[bad])
    say(f"  {name}: {int(bad.sum())} elements ({frac:.5%}) beyond the bar, worst {worst:.3g}; their Gaussians' "
        f"cancellation factors from {kap.min():.3g}; error / allowance at most {float(np.max(err[bad] / allow)):.3g}")
    assert np.all(kap >= kappa_min), f"{name}: a Gaussian without cancellation misses the bar"
    assert np.all(err[bad] <= allow), f"{name}: an element beyond its cancellation allowance"
    assert frac <= frac_cap, (name, frac)
    return frac, worst
