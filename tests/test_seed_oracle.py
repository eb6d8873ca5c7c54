"""Pins of the FP64 seeding oracle (Sec. "Dense Feature Matching": Eq. (conf)
and the two-view linear triangulation; appendix: Eq. (app-alpha-init) and the
colour median).

The pins compare the oracle with the geometry the inputs were built from
(noise-free correspondences of raycast points), with an eigen-decomposition
of the normal equations (a different library routine than the SVD), with
closed forms for the confidence mapping and for bilinear samples of linear
images, with an exposure model inverted exactly, and with a brute-force
nearest-neighbour search.  The anisotropic initialisation of Eq.
(app-sigma-init) is pinned to the normal of a known plane, the closed-form
pixel footprint on the optical axis, finite differences of the projection,
the closed-form axial scale, the viewing ray of an isolated seed, and the
rotation of every covariance under a rigid motion of the scene.
"""
import numpy as np

import oracle
from paper_2601_00705_amd import scenes

S = oracle.seeding
MAXR, MINPAR, ALO, AHI = 2.0, np.radians(0.5), 0.05, 0.95


def _run(d, **kw):
    args = dict(max_reproj=MAXR, min_parallax=MINPAR, alpha_lo=ALO, alpha_hi=AHI)
    args.update(kw)
    return S.seed(d["Ps"], d["centres"], d["images"], d["expo"], d["xr"], d["xn"], d["kappa"], **args)


def test_noise_free_matches_triangulate_the_raycast_points():
    d = scenes.seed_inputs(3, 200, noise_px=0.0, outlier_frac=0.0)
    # the generator rounds the pixel positions to float32; re-derive exact
    # float64 correspondences of the true points so the system is consistent
    X = d["X_true"]
    xr, _ = S.project(d["Ps"][0], X)
    xn = np.stack([S.project(d["Ps"][1 + k], X)[0] for k in range(d["xn"].shape[0])])
    r = S.seed(d["Ps"], d["centres"], d["images"], d["expo"], xr, xn, d["kappa"], MAXR, MINPAR, ALO, AHI)
    ok = r["angle"] >= MINPAR
    assert ok.mean() > 0.9
    assert np.all(r["valid"][ok])
    assert np.max(np.abs(r["mean"][:, ok] - X[:, ok])) < 1e-8 * np.max(np.abs(X))
    assert np.max(r["err"][ok]) < 1e-8


def test_dlt_solution_is_the_smallest_eigenvector_of_the_normal_equations():
    d = scenes.seed_inputs(4, 50)
    for i in range(50):
        xr = d["xr"][:, i].astype(np.float64)
        xn = d["xn"][0, :, i].astype(np.float64)
        X, w = S.triangulate(d["Ps"][0], d["Ps"][1], xr, xn)
        Pr, Pn = d["Ps"][0], d["Ps"][1]
        A = np.array([xr[0] * Pr[2] - Pr[0], xr[1] * Pr[2] - Pr[1], xn[0] * Pn[2] - Pn[0], xn[1] * Pn[2] - Pn[1]])
        _, vecs = np.linalg.eigh(A.T @ A)
        v = vecs[:, 0]
        Xe = v[:3] / v[3]
        assert np.allclose(X, Xe, rtol=1e-6, atol=1e-9)


def test_selection_keeps_the_lowest_error_and_rejects_outliers():
    d = scenes.seed_inputs(5, 300)
    r = _run(d)
    K = d["xn"].shape[0]
    for i in range(0, 300, 7):
        errs = []
        for k in range(K):
            X, w = S.triangulate(d["Ps"][0], d["Ps"][1 + k], d["xr"][:, i].astype(np.float64),
                                 d["xn"][k, :, i].astype(np.float64))
            yr, zr = S.project(d["Ps"][0], X[:, None])
            yn, zn = S.project(d["Ps"][1 + k], X[:, None])
            if zr[0] <= 0 or zn[0] <= 0:
                errs.append(np.inf)
                continue
            e = np.concatenate([yr[:, 0] - d["xr"][:, i], yn[:, 0] - d["xn"][k, :, i]])
            errs.append(np.sqrt(0.5 * (e @ e)))
        assert r["best"][i] == int(np.argmin(errs))
        assert np.isclose(r["err"][i], min(errs), rtol=1e-12, atol=0)
        assert r["valid"][i] == (min(errs) < MAXR and r["angle"][i] >= MINPAR)
    assert r["valid"].mean() > 0.9
    # every neighbour an outlier: only matches that happen to lie within a
    # few pixels of the epipolar line (about 4 x 2 x 2 px / 120 px of them)
    # survive the gate
    d2 = scenes.seed_inputs(6, 400, outlier_frac=1.0)
    r2 = _run(d2)
    assert r2["valid"].mean() < 0.25
    assert np.all(r2["err"][r2["valid"]] < MAXR)


def test_tie_goes_to_the_first_of_equal_hypotheses():
    d = scenes.seed_inputs(7, 40)
    # neighbour 1 duplicates neighbour 0 exactly: equal error and angle
    Ps = np.concatenate([d["Ps"][:2], d["Ps"][1:2]])
    centres = np.concatenate([d["centres"][:2], d["centres"][1:2]])
    images = [d["images"][0], d["images"][1], d["images"][1]]
    expo = np.concatenate([d["expo"][:2], d["expo"][1:2]])
    xn = np.stack([d["xn"][0], d["xn"][0]])
    kappa = np.stack([d["kappa"][0], d["kappa"][0]])
    r = S.seed(Ps, centres, images, expo, d["xr"], xn, kappa, MAXR, MINPAR, ALO, AHI)
    assert np.all(r["best"][r["valid"]] == 0)


def test_confidence_mapping_closed_form():
    d = scenes.seed_inputs(8, 30)
    for val in (0.0, 1.0, 0.25):
        kappa = np.full_like(d["kappa"], val)
        r = S.seed(d["Ps"], d["centres"], d["images"], d["expo"], d["xr"], d["xn"], kappa, MAXR, MINPAR, ALO, AHI)
        a = ALO + (AHI - ALO) * val
        assert np.allclose(r["kappa_bar"], val) and np.allclose(r["opacity_logit"], np.log(a / (1 - a)))
    r = _run(d)
    assert np.allclose(r["kappa_bar"], d["kappa"].astype(np.float64).mean(axis=0))


def test_bilinear_samples_of_a_linear_image_are_exact():
    H, W = 7, 9
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64) + 0.5
    img = np.stack([0.1 * xx + 0.2 * yy, 0.3 - 0.05 * xx, 0.02 * yy])
    for x, y in ((3.25, 2.75), (0.5, 0.5), (8.5, 6.5), (4.9, 1.1)):
        assert np.allclose(S.bilinear(img, x, y), [0.1 * x + 0.2 * y, 0.3 - 0.05 * x, 0.02 * y], atol=1e-14)
    # outside the centres the value is clamped to the border
    assert np.allclose(S.bilinear(img, 0.0, 0.0), img[:, 0, 0])


def test_colour_median_inverts_the_exposure():
    d = scenes.seed_inputs(9, 60, noise_px=0.0, outlier_frac=0.0)
    X = d["X_true"]
    xr, _ = S.project(d["Ps"][0], X)
    xn = np.stack([S.project(d["Ps"][1 + k], X)[0] for k in range(d["xn"].shape[0])])
    # every view shows the same constant colour through its exposure
    c = np.array([0.3, 0.5, 0.7])
    images = [(d["expo"][v, 0] * np.broadcast_to(c[:, None, None], im.shape) + d["expo"][v, 1]).astype(np.float64)
              for v, im in enumerate(d["images"])]
    r = S.seed(d["Ps"], d["centres"], images, d["expo"], xr, xn, d["kappa"], MAXR, MINPAR, ALO, AHI)
    assert np.allclose(r["colour"][:, r["valid"]], c[:, None], atol=1e-12)


def test_knn_scale_matches_brute_force():
    rng = np.random.default_rng(0)
    mean = rng.normal(size=(3, 400))
    mean[:, 10] = mean[:, 11]  # a duplicate point
    valid = rng.uniform(size=400) < 0.8
    valid[10] = valid[11] = True
    got = S.knn_scale(mean, valid)
    idx = np.nonzero(valid)[0]
    P = mean[:, idx].T
    D = np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(D, np.inf)
    ref = np.log(np.maximum(np.sort(D, axis=1)[:, :3].mean(axis=1), 1e-4))
    assert np.allclose(got[idx], ref, rtol=1e-12, atol=0)
    assert np.all(got[~valid] == 0.0)
    # fewer than four valid seeds: the mean over what exists
    v2 = np.zeros(400, bool)
    v2[[0, 5, 9]] = True
    got2 = S.knn_scale(mean, v2)
    P = mean[:, [0, 5, 9]].T
    D = np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(D, np.inf)
    assert np.allclose(got2[[0, 5, 9]], np.log(np.sort(D, axis=1)[:, :2].mean(axis=1)))


def _pinhole(fx, fy, R=np.eye(3), t=np.zeros(3), cx=0.0, cy=0.0):
    K = np.array([[fx, 0, cx], [0, fy, cy], [0, 0, 1.0]])
    return K @ np.hstack([R, t[:, None]])


def test_frame_fits_the_plane_of_its_neighbours():
    """Seeds on the plane n.x = 2 (a tilted wall): every seed with three or
    more neighbours in the radius gets the plane's normal, a proper
    rotation, and the covariance s_perp^2 I + (s_par^2 - s_perp^2) n n^T."""
    rng = np.random.default_rng(1)
    nrm = np.array([0.3, -0.2, 1.0])
    nrm /= np.linalg.norm(nrm)
    a = np.cross(nrm, [1.0, 0, 0])
    a /= np.linalg.norm(a)
    b = np.cross(nrm, a)
    uv = rng.uniform(-1, 1, size=(2, 300))
    mean = 2.0 * nrm[:, None] + a[:, None] * uv[0] + b[:, None] * uv[1]
    valid = np.ones(300, bool)
    err = rng.uniform(0, 3, 300)
    angle = rng.uniform(0.02, 0.5, 300)
    P = _pinhole(500.0, 500.0)
    Sigma, U, ls = S.frame_init(mean, valid, P, np.zeros(3), err, angle, radius=0.3, c_par=0.5)
    for i in range(300):
        assert abs(abs(U[i][:, 2] @ nrm) - 1.0) < 1e-12, i
        assert np.allclose(U[i].T @ U[i], np.eye(3), atol=1e-12) and np.isclose(np.linalg.det(U[i]), 1.0)
        sp, sq = np.exp(ls[0, i]), np.exp(ls[2, i])
        assert ls[0, i] == ls[1, i]
        want = sp * sp * np.eye(3) + (sq * sq - sp * sp) * np.outer(nrm, nrm)
        assert np.allclose(Sigma[i], want, rtol=0, atol=1e-12 * sq * sq)


def test_tangential_scale_is_the_pixel_footprint():
    """On the optical axis of K = diag(fx, fy, 1) the one-pixel footprint at
    depth z is an ellipse of semi-axes z / fx and z / fy: the circle of equal
    area has radius z / sqrt(fx fy).  Off the axis the Jacobian is checked
    against central differences of the projection."""
    for fx, fy, z in ((500.0, 500.0, 2.0), (300.0, 700.0, 5.5)):
        P = _pinhole(fx, fy)
        mean = np.array([[0.0], [0.0], [z]])
        _, _, ls = S.frame_init(mean, np.ones(1, bool), P, np.zeros(3), np.zeros(1), np.ones(1) * 0.3, radius=0.1)
        assert np.isclose(np.exp(ls[0, 0]), z / np.sqrt(fx * fy), rtol=1e-14)
    rng = np.random.default_rng(2)
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    R = oracle.optim.quat_to_rot(q)
    P = _pinhole(420.0, 380.0, R, np.array([0.1, -0.3, 4.0]), 320.0, 240.0)
    X = np.array([0.4, 0.2, -0.3])
    h = 1e-5
    Jfd = np.stack([(S.project(P, (X + h * e)[:, None])[0][:, 0] - S.project(P, (X - h * e)[:, None])[0][:, 0])
                    / (2 * h) for e in np.eye(3)], axis=1)
    assert np.allclose(S.projection_jacobian(P, X), Jfd, rtol=1e-7, atol=1e-6)


def test_axial_scale_and_floor():
    P = _pinhole(400.0, 400.0)
    mean = np.array([[0.0], [0.0], [4.0]])
    for err, angle, c in ((0.3, 0.1, 1.0), (2.5, 0.05, 0.7), (1.0, np.pi / 2, 2.0)):
        _, _, ls = S.frame_init(mean, np.ones(1, bool), P, np.zeros(3), np.array([err]), np.array([angle]), 0.1,
                                c_par=c)
        sp = 4.0 / 400.0
        assert np.isclose(np.exp(ls[2, 0]), c * sp * max(1.0, err) / np.sin(angle), rtol=1e-13)
    # a tiny footprint is floored, and the axial scale starts from the floor
    _, _, ls = S.frame_init(mean, np.ones(1, bool), _pinhole(1e6, 1e6), np.zeros(3), np.zeros(1),
                            np.array([np.pi / 2]), 0.1, floor=1e-4)
    assert np.allclose(np.exp(ls[:, 0]), 1e-4, rtol=1e-13)


def test_isolated_seed_takes_the_viewing_ray():
    rng = np.random.default_rng(3)
    mean = rng.normal(size=(3, 50)) * 10.0 + np.array([[0.0], [0.0], [30.0]])
    c = np.array([0.5, -0.2, 0.1])
    Sigma, U, ls = S.frame_init(mean, np.ones(50, bool), _pinhole(500.0, 500.0, t=-c), c, np.ones(50),
                                np.ones(50) * 0.2, radius=1e-3)
    for i in range(50):
        ray = (mean[:, i] - c) / np.linalg.norm(mean[:, i] - c)
        lam, V = np.linalg.eigh(Sigma[i])
        assert abs(abs(V[:, 2] @ ray) - 1.0) < 1e-10 and np.isclose(lam[2], np.exp(2 * ls[2, i]), rtol=1e-10)


def test_frame_moves_with_the_scene():
    """A rigid motion x -> Q x + s of the seeds, the camera centre and the
    projection (P -> P [Q^T, -Q^T s; 0, 1]) rotates every covariance:
    Sigma -> Q Sigma Q^T.  Invalid seeds get zeros."""
    d = scenes.seed_inputs(4, 600)
    mean = d["X_true"]
    valid = np.random.default_rng(4).uniform(size=600) < 0.9
    err = np.random.default_rng(5).uniform(0, 2, 600)
    angle = np.random.default_rng(6).uniform(0.01, 0.3, 600)
    P, c = d["Ps"][0], d["centres"][0]
    S0, _, _ = S.frame_init(mean, valid, P, c, err, angle, radius=0.4)
    q = np.random.default_rng(7).normal(size=4)
    Q = oracle.optim.quat_to_rot(q / np.linalg.norm(q))
    s = np.array([1.0, -2.0, 0.5])
    T = np.eye(4)
    T[:3, :3], T[:3, 3] = Q.T, -Q.T @ s
    S1, _, _ = S.frame_init(Q @ mean + s[:, None], valid, P @ T, Q @ c + s, err, angle, radius=0.4)
    for i in np.nonzero(valid)[0]:
        assert np.allclose(S1[i], Q @ S0[i] @ Q.T, rtol=0, atol=1e-9 * np.abs(S0[i]).max()), i
    assert np.all(S0[~valid] == 0.0)
