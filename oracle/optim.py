"""FP64 oracle of the map-maintenance steps: the Adam update with gradient
clipping and the EMA anchor, the co-visibility score, pruning and merging.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers; the product path never imports it.

Follows:
  - the appendix's optimisation settings: Adam (Kingma and Ba, Algorithm 1)
    with (beta1, beta2) = (0.9, 0.999), per-group learning rates (2e-3 for
    colour and opacity, 1e-3 for positions and rotations) and gradient norm
    clipping at 1.0;
  - Eq. (app-ema): after each mapping step the anchor of every mean moves to
    (1 - eta) anchor + eta mean;
  - Eq. (iou): IoU of the visible-pixel sets of two frames, a pixel visible
    when its accumulated opacity exceeds a threshold;
  - the pruning rule of Sec. "Insertion, Lightweight Merging, and Pruning":
    a Gaussian is removed when m_i < m_min, v_i < v_min,
    tr(Sigma_i^W) > sigma_max^2 or alpha_i < alpha_min;
  - the merging of the same section: neighbouring Gaussians with highly
    overlapping footprints and similar colours become one, with the
    visibility-weighted mean of colour and covariance.

Readings where the paper is silent:
  - epsilon = 1e-8 and the bias-corrected step of Algorithm 1; the log-scales
    take the positions' learning rate (the geometry group); every rate is an
    argument, the scheduled value of the call;
  - clipping is on the global L2 norm of all parameter gradients of the call,
    scale min(1, max_norm / (norm + 1e-6)), applied before the moments;
  - the EMA runs on the updated means;
  - accumulated opacity is 1 - T_final; the comparison 1 - T > tau is taken
    in float32, the renderer's precision; an empty union scores IoU 0;
  - tr(Sigma^W) = sum_k exp(2 log_scale_k) (Sigma = R diag(s^2) R^T), alpha =
    sigmoid(opacity_logit); the kept Gaussians keep their order;
  - merging: a pair is two mutual nearest neighbours (centre distance; each
    Gaussian merges at most once per call); the footprints overlap highly
    when the centres lie within `radius` times the smaller geometric-mean
    scale exp(mean log_scale); colours are similar when the first three
    colour rows (RGB, or SH band 0) differ by at most `colour_tol`; the
    weights are the visibilities v (equal when both are 0); mean, colour
    rows and opacity (as alpha) are weighted means as well; the merged
    covariance is split back into a rotation and scales by its eigenvectors
    and eigenvalues; the merged Gaussian takes the lower index.
"""
from __future__ import annotations

import numpy as np

PLANES = ("mean", "quat", "log_scale", "opacity_logit", "colour")


def clip_scale(grads, max_norm):
    """min(1, max_norm / (norm + 1e-6)) over all planes (1 if max_norm <= 0),
    and the norm."""
    norm = np.sqrt(sum(float((np.asarray(g, np.float64) ** 2).sum()) for g in grads.values()))
    if max_norm <= 0:
        return 1.0, norm
    return min(1.0, max_norm / (norm + 1e-6)), norm


def adam_step(params, grads, m, v, anchor, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, max_norm=1.0, ema=0.0):
    """One step.  params, grads, m, v: dicts of arrays over PLANES; lr: dict
    of rates per plane; anchor: [3][n] or None.  Returns new (params, m, v,
    anchor, norm) in float64."""
    c, norm = clip_scale(grads, max_norm)
    out_p, out_m, out_v = {}, {}, {}
    for k in PLANES:
        g = c * np.asarray(grads[k], np.float64)
        mk = beta1 * np.asarray(m[k], np.float64) + (1.0 - beta1) * g
        vk = beta2 * np.asarray(v[k], np.float64) + (1.0 - beta2) * g * g
        mhat = mk / (1.0 - beta1 ** step)
        vhat = vk / (1.0 - beta2 ** step)
        out_p[k] = np.asarray(params[k], np.float64) - lr[k] * mhat / (np.sqrt(vhat) + eps)
        out_m[k], out_v[k] = mk, vk
    new_anchor = None
    if anchor is not None:
        new_anchor = (1.0 - ema) * np.asarray(anchor, np.float64) + ema * out_p["mean"]
    return out_p, out_m, out_v, new_anchor, norm


def covis(T_key, T_frames, tau):
    """T_key [P] and T_frames [F][P] (float32 transmittance): per frame
    (intersection, union, IoU)."""
    t = np.float32(tau)
    a = (np.float32(1.0) - np.asarray(T_key, np.float32)) > t
    out = []
    for T in np.asarray(T_frames, np.float32):
        b = (np.float32(1.0) - T) > t
        inter = int(np.count_nonzero(a & b))
        uni = int(np.count_nonzero(a | b))
        out.append((inter, uni, inter / uni if uni else 0.0))
    return out


def prune_keep(m_obs, v_vis, log_scale, opacity_logit, m_min, v_min, sigma_max, alpha_min):
    """Boolean keep mask of the pruning rule."""
    ls = np.asarray(log_scale, np.float64)
    tr = np.exp(2.0 * ls).sum(axis=0)
    alpha = 1.0 / (1.0 + np.exp(-np.asarray(opacity_logit, np.float64)))
    drop = ((np.asarray(m_obs) < m_min) | (np.asarray(v_vis, np.float64) < v_min) |
            (tr > sigma_max * sigma_max) | (alpha < alpha_min))
    return ~drop


def quat_to_rot(q):
    """Rotation matrix of the unit quaternion q = (w, x, y, z) / |q|."""
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def covariance(quat, log_scale):
    """World covariance R diag(s^2) R^T of one Gaussian."""
    R = quat_to_rot(quat)
    return R @ np.diag(np.exp(2.0 * np.asarray(log_scale, np.float64))) @ R.T


def nearest_other(mean):
    """Index of each Gaussian's nearest other Gaussian (scipy's k-d tree)."""
    from scipy.spatial import cKDTree
    pts = np.asarray(mean, np.float64).T
    _, idx = cKDTree(pts).query(pts, k=2)
    return idx[:, 1]


def merge(params, v_vis, radius, colour_tol, nn=None):
    """The merging of Sec. "Insertion, Lightweight Merging, and Pruning":
    mutual nearest neighbours i < j whose centres lie within radius times the
    smaller geometric-mean scale and whose first three colour rows differ by
    at most colour_tol are replaced by one Gaussian at index i carrying the
    visibility-weighted mean of mean, colour, opacity (as alpha) and world
    covariance; j is dropped.  Returns (new params in float64, keep mask)."""
    p = {k: np.array(v, np.float64) for k, v in params.items()}
    n = p["opacity_logit"].shape[0]
    nn = nearest_other(params["mean"]) if nn is None else np.asarray(nn)
    keep = np.ones(n, bool)
    out = {k: v.copy() for k, v in p.items()}
    sbar = np.exp(p["log_scale"].mean(axis=0))
    col = p["colour"].reshape(-1, n)
    for i in range(n):
        j = int(nn[i])
        if j <= i or nn[j] != i:
            continue
        d = np.linalg.norm(p["mean"][:, i] - p["mean"][:, j])
        if not (d <= radius * min(sbar[i], sbar[j])):
            continue
        if not (np.abs(col[:3, i] - col[:3, j]).max() <= colour_tol):
            continue
        wi, wj = float(v_vis[i]), float(v_vis[j])
        if not (wi + wj > 0.0):
            wi = wj = 1.0
        W = wi + wj
        out["mean"][:, i] = (wi * p["mean"][:, i] + wj * p["mean"][:, j]) / W
        oc = out["colour"].reshape(-1, n)
        oc[:, i] = (wi * col[:, i] + wj * col[:, j]) / W
        out["opacity_logit"][i] = merged_logit(p["opacity_logit"][i], p["opacity_logit"][j], wi, wj)
        S = (wi * covariance(p["quat"][:, i], p["log_scale"][:, i]) +
             wj * covariance(p["quat"][:, j], p["log_scale"][:, j])) / W
        lam, V = np.linalg.eigh(S)
        if np.linalg.det(V) < 0:
            V[:, 0] = -V[:, 0]
        out["log_scale"][:, i] = 0.5 * np.log(lam)
        out["quat"][:, i] = rot_to_quat(V)
        keep[j] = False
    return out, keep


def merged_logit(xi, xj, wi, wj):
    """logit of the weighted mean (wi sigmoid(xi) + wj sigmoid(xj)) / (wi + wj).
    The mean a and its complement 1 - a are both formed as weighted sums of
    sigmoids (1 - sigmoid(x) = sigmoid(-x)) in the log domain, so that
    saturated opacities (|logit| beyond ~37, where a rounds to 1 in double)
    keep a finite logit log(a) - log(1 - a)."""
    with np.errstate(divide="ignore"):
        lw = np.log(np.array([wi, wj], np.float64))  # a zero weight gives -inf
    x = np.array([xi, xj], np.float64)
    log_sig = -np.logaddexp(0.0, -x)      # log sigmoid(x)
    log_sig_neg = -np.logaddexp(0.0, x)   # log sigmoid(-x) = log(1 - sigmoid(x))
    return float(np.logaddexp.reduce(lw + log_sig) - np.logaddexp.reduce(lw + log_sig_neg))


def rot_to_quat(R):
    """A unit quaternion (w, x, y, z) of the rotation matrix R (scipy)."""
    from scipy.spatial.transform import Rotation
    x, y, z, w = Rotation.from_matrix(R).as_quat()
    return np.array([w, x, y, z])
