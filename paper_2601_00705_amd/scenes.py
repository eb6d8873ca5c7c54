"""Seeded synthetic inputs for the renderer: Gaussian sets, cameras, poses.

This module holds input synthesis only -- none of the renderer's arithmetic --
and is shared by the tests, the benchmark and the CPU oracle's callers.  All
draws use NumPy's PCG64 ``default_rng(seed)`` in float64 and are cast to
float32 at the end.  Parameters are structure-of-arrays planes:

    mean [3, N], quat [4, N] (w, x, y, z), log_scale [3, N],
    opacity_logit [N], colour [3, N] (RGB) or [K, 3, N] (SH, K = (d+1)^2).

Cameras are dicts {width, height, fx, fy, cx, cy}; poses are world-to-camera
[R | t] rows (R row-major, then t), x_c = R x_w + t, stacked as [V, 12].

The workloads stand in for the paper's TUM RGB-D (640x480) and Replica
(1200x680) sequences, which are not available: a textured 6 x 3 x 5 m room
(walls plus spheres) supplies the indoor structure.  World axes: x right,
y down, z forward (the camera frame at the identity pose).
"""
from __future__ import annotations

import math

import numpy as np

ROOM_HALF = np.array([3.0, 1.5, 2.5])   # 6 x 3 x 5 m box centred at the origin
LOG_SCALE_RANGE = (math.log(0.01), math.log(0.1))
Y00 = 0.5 / math.sqrt(math.pi)          # constant SH basis function


def camera(width, height, f):
    return {"width": int(width), "height": int(height), "fx": float(f), "fy": float(f),
            "cx": width / 2.0, "cy": height / 2.0}


def identity_pose():
    return np.concatenate([np.eye(3).reshape(9), np.zeros(3)])


def pose_from_centre(centre, yaw, pitch):
    """World-to-camera pose for a camera at ``centre`` turned by yaw about the
    vertical (y) axis and pitch about its own x axis, roll 0."""
    cyw, syw, cp, sp = math.cos(yaw), math.sin(yaw), math.cos(pitch), math.sin(pitch)
    Ry = np.array([[cyw, 0, syw], [0, 1, 0], [-syw, 0, cyw]])
    Rx = np.array([[1, 0, 0], [0, cp, -sp], [0, sp, cp]])
    R_cw = Ry @ Rx
    R = R_cw.T
    t = -R @ np.asarray(centre, dtype=np.float64)
    return np.concatenate([R.reshape(9), t])


def twist_hat(xi):
    """4x4 matrix of a twist xi = (rho, omega)."""
    rho, om = np.asarray(xi[:3], float), np.asarray(xi[3:], float)
    X = np.zeros((4, 4))
    X[:3, :3] = [[0, -om[2], om[1]], [om[2], 0, -om[0]], [-om[1], om[0], 0]]
    X[:3, 3] = rho
    return X


def left_perturb(pose, xi):
    """exp(xi^) T for a [12] pose, using scipy's matrix exponential."""
    from scipy.linalg import expm
    T = np.eye(4)
    T[:3, :3] = np.asarray(pose[:9]).reshape(3, 3)
    T[:3, 3] = pose[9:]
    T2 = expm(twist_hat(xi)) @ T
    return np.concatenate([T2[:3, :3].reshape(9), T2[:3, 3]])


def random_twist(rng, trans=0.01, rot_deg=0.5):
    """Twist with |rho| = trans (m) and |omega| = rot_deg (deg), random axes."""
    a = rng.normal(size=3)
    b = rng.normal(size=3)
    return np.concatenate([trans * a / np.linalg.norm(a),
                           math.radians(rot_deg) * b / np.linalg.norm(b)])


def random_quats(rng, n):
    q = rng.normal(size=(4, n))
    return q / np.linalg.norm(q, axis=0, keepdims=True)


def _f32(d):
    return {k: np.ascontiguousarray(v, dtype=np.float32) for k, v in d.items()}


# --------------------------------------------------------------------------
# small random cloud in front of one camera

def cloud(seed, n, width, height, f, rgb=True, sh_degree=-1):
    """N Gaussians: x, y ~ U[-1, 1], depth ~ U[2, 4]; log-scales ~ U[ln .01,
    ln .1]; random unit quaternions; opacity logits ~ N(0, 1); RGB ~ U[0, 1]."""
    rng = np.random.default_rng(seed)
    mean = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 4, n)])
    p = {
        "mean": mean,
        "quat": random_quats(rng, n),
        "log_scale": rng.uniform(*LOG_SCALE_RANGE, size=(3, n)),
        "opacity_logit": rng.normal(size=n),
    }
    if sh_degree < 0:
        p["colour"] = rng.uniform(0, 1, size=(3, n))
    else:
        K = (sh_degree + 1) ** 2
        sh = rng.normal(0, 0.1, size=(K, 3, n))
        sh[0] = rng.uniform(0, 1, size=(3, n)) / Y00
        p["colour"] = sh
    return _f32(p), camera(width, height, f)


def perturb(params, seed, sigma=0.01):
    """Every parameter array plus N(0, sigma^2) noise (the target scene)."""
    rng = np.random.default_rng(seed)
    return _f32({k: v.astype(np.float64) + rng.normal(0, sigma, size=v.shape)
                 for k, v in params.items()})


def upstream_grad(seed, n_values, scale=None):
    """L1-shaped upstream gradient: random signs / n_values (or * scale)."""
    rng = np.random.default_rng(seed)
    s = rng.choice(np.array([-1.0, 1.0]), size=n_values)
    return (s * (scale if scale is not None else 1.0 / n_values)).astype(np.float32)


def track_inputs(seed, cams):
    """Inputs of the tracking loss for concatenated views (float32): a render
    rgb [sum 3 H W] in [0, 1], its final transmittance [sum H W] (a quarter
    of the pixels empty, T = 1), and an observation [sum 3 H W] that is a
    brightness-shifted, noisy copy of the render with one flat (textureless)
    rectangle per view."""
    rng = np.random.default_rng(seed)
    rgb, T, target = [], [], []
    for c in cams:
        H, W = int(c["height"]), int(c["width"])
        img = rng.uniform(0.0, 1.0, (3, H, W))
        t = np.where(rng.uniform(size=(H, W)) < 0.25, 1.0, rng.uniform(0.0, 1.0, (H, W)))
        obs = 0.85 * img + 0.06 + rng.normal(0.0, 0.05, (3, H, W))
        y0, x0 = int(rng.integers(0, H)), int(rng.integers(0, W))
        obs[:, y0:y0 + max(1, H // 3), x0:x0 + max(1, W // 3)] = rng.uniform(0.2, 0.8, (3, 1, 1))
        rgb.append(img.ravel())
        T.append(t.ravel())
        target.append(obs.ravel())
    return (np.concatenate(rgb).astype(np.float32), np.concatenate(T).astype(np.float32),
            np.concatenate(target).astype(np.float32))


# --------------------------------------------------------------------------
# textured room: 6 walls + spheres

_WALL_BASE = np.array([[0.80, 0.70, 0.60], [0.55, 0.65, 0.80], [0.70, 0.80, 0.55],
                       [0.85, 0.55, 0.50], [0.60, 0.60, 0.60], [0.75, 0.75, 0.90]])


def texture(points, base):
    """Procedural colour: base x prod over axes of (0.75 + 0.25 sin(2 pi p / 0.25))."""
    f = np.ones(points.shape[1])
    for a, ph in zip(range(3), (0.0, 1.3, 2.1)):
        f = f * (0.75 + 0.25 * np.sin(2 * np.pi * points[a] / 0.25 + ph))
    return base[:, None] * f[None, :] if base.ndim == 1 else base * f[None, :]


def _wall_samples(rng, n):
    """Area-weighted uniform points on the 6 walls; returns points and wall id."""
    hx, hy, hz = ROOM_HALF
    areas = np.array([4 * hy * hz, 4 * hy * hz, 4 * hx * hz, 4 * hx * hz, 4 * hx * hy, 4 * hx * hy])
    wall = rng.choice(6, size=n, p=areas / areas.sum())
    u1, u2 = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    P = np.zeros((3, n))
    for w in range(6):
        m = wall == w
        ax = w // 2
        sign = -1.0 if w % 2 == 0 else 1.0
        others = [a for a in range(3) if a != ax]
        P[ax, m] = sign * ROOM_HALF[ax]
        P[others[0], m] = u1[m] * ROOM_HALF[others[0]]
        P[others[1], m] = u2[m] * ROOM_HALF[others[1]]
    return P, wall


def _spheres(rng, count, avoid):
    """Sphere centres/radii inside the room, clear of the walls by 0.6 m and of
    every point in ``avoid`` by radius + 0.3 m."""
    out = []
    while len(out) < count:
        r = rng.uniform(0.15, 0.5)
        c = rng.uniform(-(ROOM_HALF - 0.6 - r), ROOM_HALF - 0.6 - r)
        if all(np.linalg.norm(c - a) >= r + 0.3 for a in avoid):
            out.append((c, r))
    return out


def _sphere_samples(rng, n, spheres):
    areas = np.array([r * r for _, r in spheres])
    which = rng.choice(len(spheres), size=n, p=areas / areas.sum())
    d = rng.normal(size=(3, n))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    C = np.stack([spheres[k][0] for k in which], axis=1)
    Rr = np.array([spheres[k][1] for k in which])
    return C + d * Rr[None, :], which


def _sphere_base(k):
    rng = np.random.default_rng(7919 + k)
    return rng.uniform(0.3, 1.0, size=3)


def room_scene(seed, n_wall, n_sphere, avoid, sh_degree=-1, n_spheres=20):
    """Gaussians on the room's walls and on ``n_spheres`` spheres.  Scales,
    quaternions and opacity logits as in ``cloud``; colour = texture at the mean
    (as SH: k00 = texture / Y00, higher bands ~ N(0, 0.05^2))."""
    rng = np.random.default_rng(seed)
    spheres = _spheres(rng, n_spheres, avoid)
    Pw, wall = _wall_samples(rng, n_wall)
    Ps, which = _sphere_samples(rng, n_sphere, spheres)
    mean = np.concatenate([Pw, Ps], axis=1)
    base = np.concatenate([_WALL_BASE[wall].T, np.stack([_sphere_base(k) for k in which], axis=1)],
                          axis=1)
    rgb = texture(mean, base)
    n = n_wall + n_sphere
    p = {
        "mean": mean,
        "quat": random_quats(rng, n),
        "log_scale": rng.uniform(*LOG_SCALE_RANGE, size=(3, n)),
        "opacity_logit": rng.normal(size=n),
    }
    if sh_degree < 0:
        p["colour"] = rgb
    else:
        K = (sh_degree + 1) ** 2
        sh = rng.normal(0, 0.05, size=(K, 3, n))
        sh[0] = rgb / Y00
        p["colour"] = sh
    return _f32(p), spheres


def random_room_poses(rng, count):
    """Camera centres ~ U(room shrunk by 0.5 m), yaw ~ U[0, 2 pi), pitch ~
    U[-20, 20] deg, roll 0."""
    poses, centres = [], []
    for _ in range(count):
        c = rng.uniform(-(ROOM_HALF - 0.5), ROOM_HALF - 0.5)
        yaw = rng.uniform(0, 2 * math.pi)
        pitch = math.radians(rng.uniform(-20, 20))
        poses.append(pose_from_centre(c, yaw, pitch))
        centres.append(c)
    return poses, centres


# --------------------------------------------------------------------------
# analytic raycast of the room (for the seeded-mapping workload)

def raycast(origin, dirs, spheres):
    """First hit of rays origin + s dirs (dirs [3, n], unit) with the room's
    spheres and walls; returns hit points [3, n] and colours [3, n]."""
    n = dirs.shape[1]
    best = np.full(n, np.inf)
    col = np.zeros((3, n))
    pts = np.zeros((3, n))
    # walls (ray starts inside the box: take the exit distance per axis)
    with np.errstate(divide="ignore", invalid="ignore"):
        for ax in range(3):
            for sign, wid in ((-1.0, 2 * ax), (1.0, 2 * ax + 1)):
                s = (sign * ROOM_HALF[ax] - origin[ax]) / dirs[ax]
                s = np.where(s > 1e-9, s, np.inf)
                m = s < best
                best = np.where(m, s, best)
                col[:, m] = _WALL_BASE[wid][:, None]
    for k, (c, r) in enumerate(spheres):
        oc = origin - c
        b = dirs.T @ oc
        disc = b * b - (oc @ oc - r * r)
        sq = np.sqrt(np.maximum(disc, 0))
        s = np.where(disc > 0, -b - sq, np.inf)
        s = np.where(s > 1e-9, s, np.inf)
        m = s < best
        best = np.where(m, s, best)
        col[:, m] = _sphere_base(k)[:, None]
    pts = origin[:, None] + dirs * best[None, :]
    return pts, texture(pts, col)


def _pixel_rays(pose, cam, px, py):
    R = pose[:9].reshape(3, 3)
    t = pose[9:]
    centre = -R.T @ t
    d_cam = np.stack([(px - cam["cx"]) / cam["fx"], (py - cam["cy"]) / cam["fy"], np.ones_like(px)])
    d = R.T @ d_cam
    return centre, d / np.linalg.norm(d, axis=0, keepdims=True)


def raycast_image(pose, cam, spheres):
    """Analytic [3, H, W] image of the room (pixel centres at +0.5)."""
    W, H = cam["width"], cam["height"]
    py, px = np.mgrid[0:H, 0:W].astype(np.float64) + 0.5
    centre, d = _pixel_rays(pose, cam, px.ravel(), py.ravel())
    _, c = raycast(centre, d, spheres)
    return c.reshape(3, H, W).astype(np.float32)


def _project_pts(pose, cam, X):
    R = pose[:9].reshape(3, 3)
    xc = R @ X + pose[9:, None]
    return np.stack([cam["fx"] * xc[0] / xc[2] + cam["cx"], cam["fy"] * xc[1] / xc[2] + cam["cy"]]), xc[2]


def _projection_matrix(pose, cam):
    K = np.array([[cam["fx"], 0, cam["cx"]], [0, cam["fy"], cam["cy"]], [0, 0, 1.0]])
    return K @ np.concatenate([pose[:9].reshape(3, 3), pose[9:, None]], axis=1)


def _dlt_batch(P1, P2, x1, x2):
    """Two-view linear triangulation (homogeneous 4x4 system, smallest right
    singular vector), float64, vectorised over points."""
    A = np.stack([x1[0][:, None] * P1[2][None, :] - P1[0][None, :],
                  x1[1][:, None] * P1[2][None, :] - P1[1][None, :],
                  x2[0][:, None] * P2[2][None, :] - P2[0][None, :],
                  x2[1][:, None] * P2[2][None, :] - P2[1][None, :]], axis=1)
    _, _, Vt = np.linalg.svd(A)
    Xh = Vt[:, -1, :]
    return (Xh[:, :3] / Xh[:, 3:4]).T


def _bilinear(img, x, y):
    C, H, W = img.shape
    x = np.clip(x - 0.5, 0, W - 1.000001)
    y = np.clip(y - 0.5, 0, H - 1.000001)
    x0, y0 = np.floor(x).astype(int), np.floor(y).astype(int)
    fx, fy = x - x0, y - y0
    x1, y1 = np.minimum(x0 + 1, W - 1), np.minimum(y0 + 1, H - 1)
    return (img[:, y0, x0] * (1 - fx) * (1 - fy) + img[:, y0, x1] * fx * (1 - fy) +
            img[:, y1, x0] * (1 - fx) * fy + img[:, y1, x1] * fx * fy)


def seed_inputs(seed, n_points, n_views=5, width=160, height=120, f=100.0, noise_px=0.5, outlier_frac=0.1):
    """Inputs of the one-shot seeding for one reference keyframe (view 0) and
    n_views - 1 neighbours: a keyframe path looking at the +z wall of the
    analytic room (baselines ~ U[5, 15] cm, +-5 deg jitter), the keyframe
    images, a per-view exposure (g, b) ~ (U[0.9, 1.1], U[-0.05, 0.05]) applied
    to the neighbours' images (the reference keeps (1, 0)), and per reference
    pixel: its position, the raycast point seen there, and per neighbour the
    point's projection perturbed by N(0, noise_px^2) (for outlier_frac of the
    matches a uniform pixel instead) with a confidence ~ U[0.6, 1] for
    inliers and U[0, 0.4] for outliers.  No triangulation happens here."""
    rng = np.random.default_rng(seed)
    cam = camera(width, height, f)
    poses, centre = [], np.array([-0.3, 0.0, 0.0])
    for k in range(n_views):
        if k:
            step = rng.normal(size=3)
            step[2] *= 0.2
            centre = centre + step / np.linalg.norm(step) * rng.uniform(0.05, 0.15)
        yaw, pitch = np.radians(rng.uniform(-5, 5)), np.radians(rng.uniform(-5, 5))
        poses.append(pose_from_centre(centre, yaw, pitch))
    centres = np.stack([-(p[:9].reshape(3, 3).T @ p[9:]) for p in poses])
    spheres = _spheres(rng, 20, list(centres))
    expo = np.stack([[1.0, 0.0]] + [[rng.uniform(0.9, 1.1), rng.uniform(-0.05, 0.05)] for _ in range(n_views - 1)])
    images = [(expo[v, 0] * raycast_image(p, cam, spheres) + expo[v, 1]).astype(np.float32)
              for v, p in enumerate(poses)]
    Ps = np.stack([_projection_matrix(p, cam) for p in poses])
    px = rng.uniform(0, width, n_points)
    py = rng.uniform(0, height, n_points)
    oc, d = _pixel_rays(poses[0], cam, px, py)
    X, _ = raycast(oc, d, spheres)
    K = n_views - 1
    xn = np.zeros((K, 2, n_points))
    kappa = np.zeros((K, n_points))
    for k in range(K):
        x2, _ = _project_pts(poses[1 + k], cam, X)
        x2 = x2 + rng.normal(0, noise_px, size=x2.shape)
        out = rng.uniform(size=n_points) < outlier_frac
        x2[0, out] = rng.uniform(0, width, out.sum())
        x2[1, out] = rng.uniform(0, height, out.sum())
        xn[k] = x2
        kappa[k] = np.where(out, rng.uniform(0.0, 0.4, n_points), rng.uniform(0.6, 1.0, n_points))
    xr = np.stack([px, py]) + rng.normal(0, noise_px, size=(2, n_points))
    return {"cams": [dict(cam) for _ in range(n_views)], "poses": np.stack(poses), "Ps": Ps, "centres": centres,
            "images": images, "expo": expo, "X_true": X, "xr": xr.astype(np.float32),
            "xn": xn.astype(np.float32), "kappa": kappa.astype(np.float32)}


def seeded_keyframes(seed, n_target, n_views=5, width=1200, height=680, f=600.0,
                     noise_px=0.5, outlier_frac=0.1, max_reproj=2.0, batch=200_000):
    """Gaussians triangulated from synthetic dense correspondences across a
    window of keyframes (the paper's one-shot seeding, as input synthesis).

    Keyframes follow a path looking at the +z wall (about 2.5 m away) with
    baselines ~ U[5, 15] cm and +-5 deg orientation jitter.  Reference pixels
    of each keyframe in turn are raycast into the analytic room, projected into
    the other keyframes, perturbed by N(0, noise_px^2) and, for outlier_frac of
    them, replaced by uniform pixels.  Each (reference, neighbour) pair is
    triangulated by the linear two-view method; the hypothesis with the lowest
    reprojection error is kept, ties going to the larger baseline angle, and
    kept only if its error is below max_reproj px and it lies in front of both
    cameras.  The first n_target survivors in generation order become
    Gaussians: isotropic scale = mean distance to the 3 nearest neighbours,
    identity rotation, opacity 0.1, colour bilinearly sampled from the
    reference image."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    cam = camera(width, height, f)
    poses, centre = [], np.array([-0.3, 0.0, 0.0])
    for k in range(n_views):
        if k:
            step = rng.normal(size=3)
            step[2] *= 0.2
            centre = centre + step / np.linalg.norm(step) * rng.uniform(0.05, 0.15)
        yaw, pitch = np.radians(rng.uniform(-5, 5)), np.radians(rng.uniform(-5, 5))
        poses.append(pose_from_centre(centre, yaw, pitch))
    centres = [-(p[:9].reshape(3, 3).T @ p[9:]) for p in poses]
    spheres = _spheres(rng, 20, centres)
    images = [raycast_image(p, cam, spheres) for p in poses]
    Ps = [_projection_matrix(p, cam) for p in poses]
    means, cols = [], []
    got, ref = 0, 0
    while got < n_target:
        r = ref % n_views
        ref += 1
        px = rng.uniform(0, width, batch)
        py = rng.uniform(0, height, batch)
        oc, d = _pixel_rays(poses[r], cam, px, py)
        X, _ = raycast(oc, d, spheres)
        best_err = np.full(batch, np.inf)
        best_ang = np.full(batch, -1.0)
        best_X = np.zeros((3, batch))
        for nb in range(n_views):
            if nb == r:
                continue
            x2, z2 = _project_pts(poses[nb], cam, X)
            x2 = x2 + rng.normal(0, noise_px, size=x2.shape)
            x1 = np.stack([px, py]) + rng.normal(0, noise_px, size=(2, batch))
            out = rng.uniform(size=batch) < outlier_frac
            x2[0, out] = rng.uniform(0, width, out.sum())
            x2[1, out] = rng.uniform(0, height, out.sum())
            Xt = _dlt_batch(Ps[r], Ps[nb], x1, x2)
            y1, d1 = _project_pts(poses[r], cam, Xt)
            y2, d2 = _project_pts(poses[nb], cam, Xt)
            err = np.sqrt(0.5 * (np.sum((y1 - x1) ** 2, axis=0) + np.sum((y2 - x2) ** 2, axis=0)))
            ok = (d1 > 0) & (d2 > 0) & np.isfinite(err)
            err = np.where(ok, err, np.inf)
            r1 = Xt - centres[r][:, None]
            r2 = Xt - centres[nb][:, None]
            cosang = np.sum(r1 * r2, axis=0) / (np.linalg.norm(r1, axis=0) * np.linalg.norm(r2, axis=0) + 1e-300)
            ang = np.arccos(np.clip(cosang, -1, 1))
            better = (err < best_err) | ((err == best_err) & (ang > best_ang))
            best_err = np.where(better, err, best_err)
            best_ang = np.where(better, ang, best_ang)
            best_X[:, better] = Xt[:, better]
        keep = best_err < max_reproj
        take = np.nonzero(keep)[0][: n_target - got]
        means.append(best_X[:, take])
        cols.append(_bilinear(images[r], px[take], py[take]))
        got += take.size
    mean = np.concatenate(means, axis=1)
    colour = np.concatenate(cols, axis=1)
    tree = cKDTree(mean.T)
    dist, _ = tree.query(mean.T, k=4)
    scale = np.maximum(dist[:, 1:].mean(axis=1), 1e-4)
    n = mean.shape[1]
    p = {
        "mean": mean,
        "quat": np.concatenate([np.ones((1, n)), np.zeros((3, n))]),
        "log_scale": np.repeat(np.log(scale)[None, :], 3, axis=0),
        "opacity_logit": np.full(n, math.log(0.1 / 0.9)),
        "colour": colour,
    }
    return _f32(p), [dict(cam) for _ in range(n_views)], np.stack(poses), images, spheres


# --------------------------------------------------------------------------
# the five workloads

def workload(index, seed=None):
    """Returns dict(params, cams, poses, targets or target_poses, pose_only,
    sh_degree, name).  Sizes follow the five benchmark configurations.
    Parameters and poses are float32 (the renderer's input precision), so
    that every consumer sees the same inputs."""
    return _pose_f32(_workload(index, seed))


def _pose_f32(w):
    for k in ("poses", "target_poses"):
        if k in w:
            w[k] = np.ascontiguousarray(w[k], dtype=np.float32)
    return w


def _workload(index, seed=None):
    if index == 0:
        s = 1000 if seed is None else seed
        params, cam = cloud(s, 2000, 64, 48, 50.0)
        return {"name": "cloud-2k-64x48", "params": params, "cams": [cam],
                "poses": identity_pose()[None, :], "target_params": perturb(params, s + 1000),
                "sh_degree": -1, "pose_only": np.zeros(1, np.uint8)}
    if index == 1:
        s = 1001 if seed is None else seed
        params, _ = room_scene(s, 80_000, 20_000, avoid=[np.zeros(3)])
        pose = identity_pose()
        tgt = left_perturb(pose, random_twist(np.random.default_rng(s + 1000)))
        return {"name": "room-100k-640x480", "params": params, "cams": [camera(640, 480, 525.0)],
                "poses": pose[None, :], "target_poses": tgt[None, :], "sh_degree": -1,
                "pose_only": np.zeros(1, np.uint8)}
    if index == 2:
        s = 1002 if seed is None else seed
        params, cams, poses, images, _ = seeded_keyframes(s, 500_000)
        return {"name": "seeded-500k-5x1200x680", "params": params, "cams": cams, "poses": poses,
                "targets": images, "sh_degree": -1, "pose_only": np.zeros(5, np.uint8)}
    if index == 3:
        s = 1003 if seed is None else seed
        rng = np.random.default_rng(s)
        poses, centres = random_room_poses(rng, 10)
        cams = ([camera(640, 480, 525.0)] * 4 + [camera(1200, 680, 600.0)] * 4 +
                [camera(320, 240, 262.5)] * 2)
        params, _ = room_scene(s + 7, 800_000, 200_000, avoid=centres)
        trng = np.random.default_rng(s + 1000)
        tgt = np.stack([left_perturb(p, random_twist(trng)) for p in poses])
        return {"name": "window-1M-10views", "params": params, "cams": [dict(c) for c in cams],
                "poses": np.stack(poses), "target_poses": tgt, "sh_degree": -1,
                "pose_only": np.zeros(10, np.uint8)}
    if index == 4:
        s = 1004 if seed is None else seed
        rng = np.random.default_rng(s)
        poses, centres = random_room_poses(rng, 36)
        cams = [camera(1920, 1080, 1000.0)] * 4 + [camera(640, 480, 525.0)] * 32
        params, _ = room_scene(s + 7, 2_400_000, 600_000, avoid=centres, sh_degree=3)
        trng = np.random.default_rng(s + 1000)
        tgt = np.stack([left_perturb(p, random_twist(trng)) for p in poses])
        pose_only = np.array([0] * 4 + [1] * 32, dtype=np.uint8)
        return {"name": "track-map-3M-sh3-36views", "params": params, "cams": [dict(c) for c in cams],
                "poses": np.stack(poses), "target_poses": tgt, "sh_degree": 3,
                "pose_only": pose_only}
    raise ValueError(index)
