"""Brute-force NumPy forward renderer -- TEST INFRASTRUCTURE ONLY.

A second forward written independently of ``gsr_oracle.c`` and used to pin
it on tiny inputs: no tiles and no rectangles; for every pixel every live
Gaussian is evaluated, the ones whose alpha clears alpha_min are ordered by
(camera depth rounded to float32, index) and composited with Eq. (alpha).  The rotation of a
Gaussian is built by rotating the basis vectors with the Hamilton product
q v q*, not from the closed-form matrix the C code uses.

Follows Sec. "Gaussian Splatting Representation", Eq. (proj) and Eq. (alpha),
and the appendix's Sigma_W = R diag(s^2) R^T parameterisation.
"""
from __future__ import annotations

import numpy as np


def _hamilton(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([
        w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
        w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
        w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
        w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2,
    ])


def _rotation(q):
    """Columns are the images of e_x, e_y, e_z under v -> q v q*."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q)
    qc = q * np.array([1.0, -1.0, -1.0, -1.0])
    cols = []
    for e in np.eye(3):
        cols.append(_hamilton(_hamilton(q, np.concatenate([[0.0], e])), qc)[1:])
    return np.stack(cols, axis=1)


def render(params, cam, pose, cfg):
    """Returns (rgb [3,H,W], T_final [H,W], n_blend [H,W]) for one view.
    ``cfg`` needs z_near, dilation, alpha_min, alpha_max, T_min, bg; RGB only."""
    mean = np.asarray(params["mean"], dtype=np.float64)
    quat = np.asarray(params["quat"], dtype=np.float64)
    ls = np.asarray(params["log_scale"], dtype=np.float64)
    lam = np.asarray(params["opacity_logit"], dtype=np.float64)
    col = np.asarray(params["colour"], dtype=np.float64)
    n = lam.shape[0]
    pose = np.asarray(pose, dtype=np.float64).reshape(12)
    Rc, t = pose[:9].reshape(3, 3), pose[9:]
    fx, fy, cx, cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    W, H = int(cam["width"]), int(cam["height"])

    live, u, v, inv, opac, depth = [], [], [], [], [], []
    for i in range(n):
        Rq = _rotation(quat[:, i])
        L = Rq @ np.diag(np.exp(ls[:, i]))
        Sw = L @ L.T
        mc = Rc @ mean[:, i] + t
        x, y, z = mc
        ok = z > cfg.z_near
        o = 1.0 / (1.0 + np.exp(-lam[i]))
        if ok:
            J = np.array([[fx / z, 0.0, -fx * x / z ** 2], [0.0, fy / z, -fy * y / z ** 2]])
            S2 = J @ Rc @ Sw @ Rc.T @ J.T + cfg.dilation * np.eye(2)
            ok = np.linalg.det(S2) > 0
        if ok:
            live.append(i)
            u.append(fx * x / z + cx)
            v.append(fy * y / z + cy)
            inv.append(np.linalg.inv(S2))
            opac.append(o)
            depth.append(z)
    live = np.array(live, dtype=np.int64)
    rgb = np.zeros((3, H, W))
    T_out = np.ones((H, W))
    nb = np.zeros((H, W), dtype=np.int32)
    if live.size == 0:
        rgb += np.asarray(cfg.bg, dtype=np.float64)[:, None, None]
        return rgb, T_out, nb
    u, v, inv, opac, depth = map(np.asarray, (u, v, inv, opac, depth))
    # by the float32-rounded depth (the precision of the ordering key), then index
    order = np.lexsort((live, depth.astype(np.float32)))
    for py in range(H):
        for px in range(W):
            d = np.stack([px + 0.5 - u, py + 0.5 - v], axis=1)
            q = np.einsum("ni,nij,nj->n", d, inv, d)
            a_raw = opac * np.exp(-0.5 * q)
            alpha = np.minimum(cfg.alpha_max, a_raw)
            T, C, cnt = 1.0, np.zeros(3), 0
            for k in order:
                if alpha[k] < cfg.alpha_min:
                    continue
                if T * (1.0 - alpha[k]) < cfg.T_min:
                    break
                C += col[:, live[k]] * alpha[k] * T
                T *= 1.0 - alpha[k]
                cnt += 1
            rgb[:, py, px] = C + T * np.asarray(cfg.bg, dtype=np.float64)
            T_out[py, px] = T
            nb[py, px] = cnt
    return rgb, T_out, nb
