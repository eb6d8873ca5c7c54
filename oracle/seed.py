"""FP64 oracle of the one-shot Gaussian seeding from dense correspondences.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers; the product path never imports it.

Follows Sec. "Dense Feature Matching" and the appendix's initialisation:
  - Eq. (conf): the aggregated confidence of a reference pixel is the mean of
    its per-neighbour confidences;
  - "Multi-view Triangulation": for every neighbour, the two-view linear
    system A X = 0 (rows x P^3 - P^1 and y P^3 - P^2 of both views), solved by
    the right singular vector of the smallest singular value (numpy's SVD,
    double precision), dehomogenised; among the neighbours the hypothesis with
    the lowest reprojection error is kept, ties going to the larger baseline
    angle; candidates with a large reprojection error or a small parallax are
    rejected;
  - Eq. (app-alpha-init): opacity alpha_lo + (alpha_hi - alpha_lo) kappa_bar;
  - colour: the median of bilinear samples over the supporting views, after
    the per-view exposure correction.

Readings where the paper is silent:
  - the reprojection error of a hypothesis is the RMS of its two reprojection
    distances (reference and neighbour), sqrt((|e_r|^2 + |e_n|^2) / 2);
  - a hypothesis behind either camera (depth <= 0) or with a zero fourth
    homogeneous coordinate is no candidate;
  - the baseline angle is the angle at X between the rays to the two camera
    centres; a kept point needs error < max_reproj and angle >= min_parallax
    (the rejection is applied to the selected hypothesis), and a position
    representable in float32 (the Gaussian layout);
  - supporting views: the reference view and every neighbour whose matched
    pixel lies within max_reproj of the kept point's projection;
  - a sample is bilinear between pixel centres (pixel (i, j) holds the value
    at (i + 1/2, j + 1/2)), clamped to the border; the exposure correction
    inverts the tracking model I = g I_hat + b: c = (I - b) / g;
  - the median of an even number of samples is the mean of the two middle
    ones;
  - opacity_logit = log(alpha / (1 - alpha));
  - scale (the workload's stated recipe, standing in for the plane-fit
    anisotropic initialisation): isotropic, the mean distance to the 3
    nearest other kept seeds (fewer if fewer exist; 0 neighbours gives the
    floor); log_scale = log(max(that, floor)) on all three axes.
"""
from __future__ import annotations

import numpy as np


def project(P, X):
    """Pixel position and depth of world points X [3][m] under P [3][4]."""
    Xh = np.vstack([X, np.ones((1, X.shape[1]))])
    y = P @ Xh
    return y[:2] / y[2], y[2]


def triangulate(Pr, Pn, xr, xn):
    """Two-view linear triangulation of one point: (X [3], w) where w is the
    fourth homogeneous coordinate of the unit null vector (X undefined if w = 0)."""
    A = np.array([xr[0] * Pr[2] - Pr[0],
                  xr[1] * Pr[2] - Pr[1],
                  xn[0] * Pn[2] - Pn[0],
                  xn[1] * Pn[2] - Pn[1]], dtype=np.float64)
    _, _, Vt = np.linalg.svd(A)
    Xh = Vt[-1]
    if Xh[3] == 0.0:
        return None, 0.0
    return Xh[:3] / Xh[3], Xh[3]


def bilinear(img, x, y):
    """img [3][H][W]; sample at pixel position (x, y), pixel centres at +1/2."""
    _, H, W = img.shape
    fx = min(max(x - 0.5, 0.0), W - 1.0)
    fy = min(max(y - 0.5, 0.0), H - 1.0)
    x0, y0 = int(np.floor(fx)), int(np.floor(fy))
    x1, y1 = min(x0 + 1, W - 1), min(y0 + 1, H - 1)
    ax, ay = fx - x0, fy - y0
    img = np.asarray(img, np.float64)
    return (img[:, y0, x0] * (1 - ax) * (1 - ay) + img[:, y0, x1] * ax * (1 - ay) +
            img[:, y1, x0] * (1 - ax) * ay + img[:, y1, x1] * ax * ay)


def seed_point(Ps, centres, images, expo, xr, xn, kappa, max_reproj, min_parallax, alpha_lo, alpha_hi):
    """One reference pixel.  Ps[0], centres[0], images[0]: reference view;
    [1 + k]: neighbour k.  xr [2], xn [K][2], kappa [K]."""
    K = len(xn)
    best = None  # (err, angle, k, X)
    for k in range(K):
        X, w = triangulate(Ps[0], Ps[1 + k], xr, xn[k])
        if X is None:
            continue
        yr, dr = project(Ps[0], X[:, None])
        yn, dn = project(Ps[1 + k], X[:, None])
        if not (dr[0] > 0.0 and dn[0] > 0.0):
            continue
        er = yr[:, 0] - xr
        en = yn[:, 0] - xn[k]
        err = np.sqrt(0.5 * (er @ er + en @ en))
        a = X - centres[0]
        b = X - centres[1 + k]
        c = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        ang = np.arccos(min(max(c, -1.0), 1.0))
        if best is None or err < best[0] or (err == best[0] and ang > best[1]):
            best = (err, ang, k, X)
    kbar = float(np.mean(kappa))
    alpha = alpha_lo + (alpha_hi - alpha_lo) * kbar
    out = {"kappa_bar": kbar, "opacity_logit": float(np.log(alpha / (1.0 - alpha))),
           "valid": False, "best": -1, "err": np.inf, "angle": 0.0, "mean": np.zeros(3), "colour": np.zeros(3)}
    if best is None:
        return out
    err, ang, k, X = best
    out.update(best=k, err=err, angle=ang, mean=X)
    if not (err < max_reproj and ang >= min_parallax and np.all(np.isfinite(X.astype(np.float32)))):
        return out
    out["valid"] = True
    samples = []
    for v in range(K + 1):
        if v == 0:
            pos = xr
        else:
            y, _ = project(Ps[v], X[:, None])
            if np.linalg.norm(y[:, 0] - xn[v - 1]) >= max_reproj:
                continue
            pos = xn[v - 1]
        s = bilinear(images[v], pos[0], pos[1])
        g, b = expo[v]
        samples.append((s - b) / g)
    out["colour"] = np.median(np.array(samples), axis=0)
    return out


def seed(Ps, centres, images, expo, xr, xn, kappa, max_reproj, min_parallax, alpha_lo, alpha_hi):
    """All points: xr [2][n], xn [K][2][n], kappa [K][n].  Returns per-point
    arrays (float64): valid [n] bool, best [n], err [n], angle [n],
    kappa_bar [n], opacity_logit [n], mean [3][n], colour [3][n]."""
    n = xr.shape[1]
    K = xn.shape[0]
    keys = ("valid", "best", "err", "angle", "kappa_bar", "opacity_logit")
    res = {k: np.zeros(n) for k in keys}
    res["valid"] = np.zeros(n, bool)
    res["best"] = np.zeros(n, np.int64)
    res["mean"] = np.zeros((3, n))
    res["colour"] = np.zeros((3, n))
    for i in range(n):
        o = seed_point(Ps, centres, images, expo, xr[:, i].astype(np.float64),
                       xn[:, :, i].astype(np.float64), kappa[:, i].astype(np.float64),
                       max_reproj, min_parallax, alpha_lo, alpha_hi)
        for k in keys:
            res[k][i] = o[k]
        res["mean"][:, i] = o["mean"]
        res["colour"][:, i] = o["colour"]
    return res


def knn_scale(mean, valid, k=3, floor=1e-4):
    """Isotropic log-scale from the mean distance to the k nearest other valid
    seeds (scipy's k-d tree), for the valid seeds; 0 for the others."""
    from scipy.spatial import cKDTree
    mean = np.asarray(mean, np.float64)
    idx = np.nonzero(valid)[0]
    out = np.zeros(mean.shape[1])
    if idx.size == 0:
        return out
    pts = mean[:, idx].T
    m = min(k, idx.size - 1)
    if m == 0:
        out[idx] = np.log(floor)
        return out
    d, _ = cKDTree(pts).query(pts, k=m + 1)
    d = np.asarray(d).reshape(idx.size, m + 1)
    out[idx] = np.log(np.maximum(d[:, 1:].mean(axis=1), floor))
    return out
