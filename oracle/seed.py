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
  - scale (the workload's stated recipe): isotropic, the mean distance to
    the 3 nearest other kept seeds (fewer if fewer exist; 0 neighbours gives
    the floor); log_scale = log(max(that, floor)) on all three axes;
  - the anisotropic initialisation of Eq. (app-sigma-init), frame_init:
    the plane is fitted to the kept seeds within `radius` of the seed (the
    seed included) by the eigen-decomposition of their scatter about their
    mean: the normal v is the eigenvector of the smallest eigenvalue, t1
    that of the largest, t2 = v x t1; with fewer than three such seeds the
    normal is the reference viewing ray (X - c) / |X - c|.  The tangential
    scale is the radius of the circle of equal area to the one-pixel
    footprint back-projected through the reference projection's Jacobian J
    (2 x 3, world to pixels, at X): s_perp = det(J J^T)^(-1/4).  The axial
    scale is s_par = c_par s_perp max(1, err) / max(sin angle, 1e-6) (err
    the kept hypothesis' reprojection error in pixels, angle its baseline
    angle, c_par the calibration): the lateral uncertainty of one pixel, or
    of the residual when larger, stretched by the inverse parallax.  Both
    scales are floored like the isotropic one.
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


def projection_jacobian(P, X):
    """2 x 3 Jacobian of the pixel position under P [3][4] with respect to
    the world point X [3]."""
    Xh = np.append(np.asarray(X, np.float64), 1.0)
    w = P[2] @ Xh
    u, v = (P[0] @ Xh) / w, (P[1] @ Xh) / w
    return np.stack([(P[0, :3] - u * P[2, :3]) / w, (P[1, :3] - v * P[2, :3]) / w])


def _completion(v):
    """A unit vector perpendicular to the unit vector v."""
    a = np.zeros(3)
    a[np.argmin(np.abs(v))] = 1.0
    t = np.cross(v, a)
    return t / np.linalg.norm(t)


def frame_init(mean, valid, P_ref, centre_ref, err, angle, radius, c_par=1.0, floor=1e-4, only=None):
    """Eq. (app-sigma-init) for every kept seed (or the kept seeds among the
    indices `only`): returns (Sigma [n][3][3], frame [n][3][3] with columns
    (t1, t2, v), log_scale [3][n]) in float64; zeros for the others.
    mean [3][n], valid [n], err and angle [n] as written by the
    triangulation; P_ref [3][4] and centre_ref [3] of the reference
    keyframe."""
    from scipy.spatial import cKDTree
    X = np.asarray(mean, np.float64)
    n = X.shape[1]
    keep = np.asarray(valid) != 0
    idx = np.nonzero(keep)[0]
    pts = X[:, idx].T
    tree = cKDTree(pts) if idx.size else None
    P = np.asarray(P_ref, np.float64)
    Sigma = np.zeros((n, 3, 3))
    frame = np.zeros((n, 3, 3))
    ls = np.zeros((3, n))
    ask = np.ones(n, bool) if only is None else np.isin(np.arange(n), only)
    for k, i in enumerate(idx):
        if not ask[i]:
            continue
        nb = tree.query_ball_point(pts[k], radius)
        if len(nb) >= 3:
            Q = pts[nb]
            D = Q - Q.mean(axis=0)
            lam, V = np.linalg.eigh(D.T @ D)
            v, t1 = V[:, 0], V[:, 2]
        else:
            v = X[:, i] - np.asarray(centre_ref, np.float64)
            v = v / np.linalg.norm(v)
            t1 = _completion(v)
        U = np.stack([t1, np.cross(v, t1), v], axis=1)
        J = projection_jacobian(P, X[:, i])
        s_perp = max(np.linalg.det(J @ J.T) ** -0.25, floor)
        s_par = max(c_par * s_perp * max(1.0, float(err[i])) / max(np.sin(float(angle[i])), 1e-6), floor)
        Sigma[i] = U @ np.diag([s_perp ** 2, s_perp ** 2, s_par ** 2]) @ U.T
        frame[i] = U
        ls[:, i] = np.log([s_perp, s_perp, s_par])
    return Sigma, frame, ls
