"""Pins of the FP64 map-maintenance oracle: the Adam step against PyTorch's
own Adam and gradient clipping (a library routine), its closed-form first
step, the EMA anchor's limits; the co-visibility counts against scikit-learn's
Jaccard score and set identities; the pruning rule against a per-Gaussian
evaluation through the explicit covariance R diag(s^2) R^T; merging against
a copy of itself, a closed-form weighted covariance and its conditions."""
import numpy as np
import pytest
import torch

from oracle import optim as O


def _problem(rng, n, colour_rows=3):
    shapes = {"mean": (3, n), "quat": (4, n), "log_scale": (3, n), "opacity_logit": (n,),
              "colour": (colour_rows, n)}
    p = {k: rng.normal(size=s) for k, s in shapes.items()}
    return p, shapes


LR = {"mean": 1e-3, "quat": 1e-3, "log_scale": 1e-3, "opacity_logit": 2e-3, "colour": 2e-3}


@pytest.mark.parametrize("max_norm", [1.0, 0.0, 1e3])
def test_adam_matches_torch(max_norm):
    rng = np.random.default_rng(0)
    n = 50
    p, shapes = _problem(rng, n)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    opt = torch.optim.Adam([{"params": [tp[k]], "lr": LR[k]} for k in O.PLANES], betas=(0.9, 0.999), eps=1e-8)
    m = {k: np.zeros(s) for k, s in shapes.items()}
    v = {k: np.zeros(s) for k, s in shapes.items()}
    cur = {k: x.copy() for k, x in p.items()}
    for step in range(1, 4):
        g = {k: rng.normal(size=s) * 3.0 for k, s in shapes.items()}
        for k in O.PLANES:
            tp[k].grad = torch.tensor(g[k])
        if max_norm > 0:
            torch.nn.utils.clip_grad_norm_([tp[k] for k in O.PLANES], max_norm)
        opt.step()
        cur, m, v, _, _ = O.adam_step(cur, g, m, v, None, LR, step, max_norm=max_norm)
        for k in O.PLANES:
            assert np.allclose(cur[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-14), (step, k)


def test_first_step_closed_form():
    """m = v = 0 at t = 1 without clipping: p - lr g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    p, shapes = _problem(rng, 20, colour_rows=48)
    g = {k: rng.normal(size=s) for k, s in shapes.items()}
    z = {k: np.zeros(s) for k, s in shapes.items()}
    out, m1, v1, _, _ = O.adam_step(p, g, z, z, None, LR, 1, max_norm=0.0)
    for k in O.PLANES:
        assert np.allclose(out[k], p[k] - LR[k] * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-14, atol=1e-15)
        assert np.allclose(m1[k], 0.1 * g[k]) and np.allclose(v1[k], 0.001 * g[k] ** 2)


def test_clipping_bounds_the_first_moment():
    rng = np.random.default_rng(2)
    p, shapes = _problem(rng, 30)
    g = {k: rng.normal(size=s) * 100.0 for k, s in shapes.items()}
    z = {k: np.zeros(s) for k, s in shapes.items()}
    _, m1, _, _, norm = O.adam_step(p, g, z, z, None, LR, 1, max_norm=1.0)
    assert norm > 100.0
    mnorm = np.sqrt(sum((m1[k] ** 2).sum() for k in O.PLANES))
    assert np.isclose(mnorm, 0.1 * 1.0 * norm / (norm + 1e-6), rtol=1e-12)


def test_ema_anchor_limits():
    rng = np.random.default_rng(3)
    p, shapes = _problem(rng, 10)
    g = {k: rng.normal(size=s) for k, s in shapes.items()}
    z = {k: np.zeros(s) for k, s in shapes.items()}
    anchor = rng.normal(size=(3, 10))
    out, _, _, a1, _ = O.adam_step(p, g, z, z, anchor, LR, 1, ema=1.0)
    assert np.array_equal(a1, out["mean"])
    _, _, _, a0, _ = O.adam_step(p, g, z, z, anchor, LR, 1, ema=0.0)
    assert np.array_equal(a0, anchor)
    _, _, _, a, _ = O.adam_step(p, g, z, z, anchor, LR, 1, ema=0.25)
    assert np.allclose(a, 0.75 * anchor + 0.25 * out["mean"], rtol=1e-15)


def test_covisibility_counts():
    from sklearn.metrics import jaccard_score
    rng = np.random.default_rng(4)
    P = 997
    key = rng.uniform(size=P).astype(np.float32)
    frames = rng.uniform(size=(4, P)).astype(np.float32)
    frames[1] = key                    # identical frame
    frames[2] = 1.0                    # nothing visible
    tau = 0.3
    res = O.covis(key, frames, tau)
    a = (1.0 - key) > tau
    for f, (inter, uni, iou) in enumerate(res):
        b = (1.0 - frames[f]) > tau
        assert inter + uni == a.sum() + b.sum()
        if uni:
            assert np.isclose(iou, jaccard_score(a, b))
    assert res[1][2] == 1.0
    assert res[2] == (0, int(a.sum()), 0.0)
    empty = O.covis(np.ones(5, np.float32), np.ones((1, 5), np.float32), tau)
    assert empty == [(0, 0, 0.0)]


def _rot(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def test_prune_rule_against_explicit_covariance():
    rng = np.random.default_rng(5)
    n = 400
    quat = rng.normal(size=(4, n))
    ls = rng.uniform(-3, 0.5, size=(3, n))
    op = rng.normal(size=n) * 3
    m_obs = rng.integers(0, 6, size=n)
    v_vis = rng.uniform(0, 2, size=n)
    keep = O.prune_keep(m_obs, v_vis, ls, op, m_min=2, v_min=0.3, sigma_max=1.5, alpha_min=0.05)
    for i in range(n):
        R = _rot(quat[:, i])
        S = R @ np.diag(np.exp(2 * ls[:, i])) @ R.T
        alpha = 1 / (1 + np.exp(-op[i]))
        want = not (m_obs[i] < 2 or v_vis[i] < 0.3 or np.trace(S) > 1.5 ** 2 or alpha < 0.05)
        assert keep[i] == want, i
    assert 0 < keep.sum() < n


def _pair_params(rng, n=6):
    p = {"mean": rng.normal(size=(3, n)) * 10.0, "quat": rng.normal(size=(4, n)),
         "log_scale": rng.uniform(-1, 0, size=(3, n)), "opacity_logit": rng.normal(size=n),
         "colour": rng.uniform(size=(3, n))}
    return p


def test_merging_a_gaussian_with_its_copy_returns_it():
    rng = np.random.default_rng(10)
    p = _pair_params(rng)
    for k in p:
        p[k][..., 1] = p[k][..., 0]
    p["mean"][:, 1] += 1e-6  # not identical positions: a unique nearest neighbour
    out, keep = O.merge(p, np.ones(6), radius=0.5, colour_tol=0.1)
    assert keep.tolist() == [True, False, True, True, True, True]
    S0 = O.covariance(p["quat"][:, 0], p["log_scale"][:, 0])
    assert np.allclose(O.covariance(out["quat"][:, 0], out["log_scale"][:, 0]), S0, rtol=1e-10, atol=1e-14)
    assert np.allclose(out["colour"][:, 0], p["colour"][:, 0]) and np.isclose(out["opacity_logit"][0],
                                                                               p["opacity_logit"][0])
    for k in p:  # the others untouched
        assert np.array_equal(out[k][..., 2:], p[k][..., 2:])


def test_merged_covariance_and_weights():
    """Two axis-aligned Gaussians, visibilities 1 and 3: every merged
    quantity is the 1:3 weighted mean (covariance through R diag(s^2) R^T,
    opacity as alpha)."""
    rng = np.random.default_rng(11)
    p = _pair_params(rng, 4)
    p["mean"][:, 1] = p["mean"][:, 0] + np.array([0.01, 0.0, 0.0])
    p["quat"][:, :2] = np.array([[1.0, 0, 0, 0], [1.0, 0, 0, 0]]).T
    p["log_scale"][:, 0] = np.log([0.1, 0.2, 0.3])
    p["log_scale"][:, 1] = np.log([0.3, 0.2, 0.1])
    p["colour"][:, 1] = p["colour"][:, 0] + 0.01
    out, keep = O.merge(p, np.array([1.0, 3.0, 1.0, 1.0]), radius=1.0, colour_tol=0.05)
    assert keep.tolist() == [True, False, True, True]
    want = np.diag((np.array([0.1, 0.2, 0.3]) ** 2 + 3 * np.array([0.3, 0.2, 0.1]) ** 2) / 4)
    assert np.allclose(O.covariance(out["quat"][:, 0], out["log_scale"][:, 0]), want, rtol=1e-12, atol=1e-15)
    assert np.allclose(out["mean"][:, 0], (p["mean"][:, 0] + 3 * p["mean"][:, 1]) / 4)
    a = lambda z: 1 / (1 + np.exp(-z))  # noqa: E731
    assert np.isclose(a(out["opacity_logit"][0]), (a(p["opacity_logit"][0]) + 3 * a(p["opacity_logit"][1])) / 4)


def test_merge_conditions():
    rng = np.random.default_rng(12)
    p = _pair_params(rng, 3)
    p["mean"][:, 1] = p["mean"][:, 0] + 0.05
    p["log_scale"][:, :2] = np.log(0.1)
    p["colour"][:, 1] = p["colour"][:, 0]
    # distance 0.0866 vs radius 0.5 x 0.1: too far
    assert O.merge(p, np.ones(3), radius=0.5, colour_tol=0.1)[1].all()
    assert not O.merge(p, np.ones(3), radius=1.0, colour_tol=0.1)[1].all()
    p["colour"][0, 1] += 0.2  # colours too different
    assert O.merge(p, np.ones(3), radius=1.0, colour_tol=0.1)[1].all()
    # a nearest neighbour that is not mutual merges nothing
    q = {k: v.copy() for k, v in _pair_params(rng, 3).items()}
    q["mean"][:, 0] = 0.0
    q["mean"][:, 1] = [1.0, 0, 0]
    q["mean"][:, 2] = [1.5, 0, 0]   # 0 -> 1, 1 -> 2, 2 -> 1: only (1, 2) is mutual
    q["log_scale"][:] = np.log(10.0)
    q["colour"][:] = 0.5
    _, keep = O.merge(q, np.ones(3), radius=1.0, colour_tol=0.1)
    assert keep.tolist() == [True, True, False]


def test_merged_opacity_of_saturated_logits_is_finite():
    """Opacity logits of 40 and 45 (alpha rounds to 1 in double): the merged
    logit is log(a / (1 - a)) with 1 - a = (e^-40 + 3 e^-45) / 4 to double
    precision, not +inf; two logits of -40 merge to -40 + log((1 + 3) / 4);
    a zero weight returns the other Gaussian's logit."""
    rng = np.random.default_rng(13)
    p = _pair_params(rng, 3)
    p["mean"][:, 1] = p["mean"][:, 0] + 0.001
    p["colour"][:, 1] = p["colour"][:, 0]
    p["log_scale"][:, :2] = np.log(0.1)
    p["opacity_logit"][:2] = [40.0, 45.0]
    out, keep = O.merge(p, np.array([1.0, 3.0, 1.0]), radius=1.0, colour_tol=0.1)
    assert keep.tolist() == [True, False, True]
    want = -np.log((np.exp(-40.0) + 3 * np.exp(-45.0)) / 4)  # 1 - a, with a within 1e-17 of 1
    assert np.isfinite(out["opacity_logit"][0]) and abs(out["opacity_logit"][0] - want) <= 1e-12 * want
    p["opacity_logit"][:2] = [-40.0, -40.0]
    out, _ = O.merge(p, np.array([1.0, 3.0, 1.0]), radius=1.0, colour_tol=0.1)
    assert abs(out["opacity_logit"][0] + 40.0) <= 1e-12
    assert O.merged_logit(40.0, -3.0, 2.0, 0.0) == 40.0
    assert abs(O.merged_logit(0.7, -0.2, 0.0, 5.0) + 0.2) <= 1e-15
