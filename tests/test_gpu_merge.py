"""Parity of the GPU merging (gsr_nearest, gsr_merge, gsr_keep_list,
gsr_compact through the C ABI) with the FP64 oracle.

Bar.  Nearest neighbour: an index, compared exactly wherever the oracle's
nearest and second-nearest distances differ by more than 1e-9 relative (the
GPU compares squared distances of the FP32 centres in double, ties to the
lower index; the oracle's k-d tree leaves the order of ties open);
elsewhere the GPU's pick must lie within 1e-9 relative of the nearest
distance.  Merge decisions
are taken in double from the same FP32 inputs on both sides, so the keep
masks are equal (the test asserts that no pair lies within 1e-9 of a
threshold).  The merged columns are FP64 results rounded once to FP32: mean,
colour and opacity logit within 1e-6 relative (plus 1e-7 absolute); the
world covariance rebuilt from the FP32 quaternion and log-scales within
1e-5 of its largest entry (the eigenvectors of a near-degenerate covariance
are not unique, the covariance is); unmerged columns are bitwise copies.
"""
import numpy as np
import pytest
import torch

from oracle import optim as O

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2601_00705_amd import maintain

PLANES = O.PLANES


def say(msg):
    print(msg, flush=True)


def _cloud(seed, n_base, n_pairs, colour_rows=3, box=5.0, offset=0.01, cdiff=0.06, zero_pairs=20):
    """Isolated Gaussians in a cube plus close partners of some of them
    (offset ~ N(0, offset^2) per axis, colour shifted by up to cdiff),
    shuffled; visibilities in [0, 2), both zero for a few pairs."""
    rng = np.random.default_rng(seed)
    base = rng.uniform(-box, box, size=(3, n_base))
    pick = rng.choice(n_base, n_pairs, replace=False)
    mean = np.concatenate([base, base[:, pick] + rng.normal(size=(3, n_pairs)) * offset], 1)
    n = n_base + n_pairs
    colour = rng.uniform(0, 1, size=(colour_rows, n_base))
    colour = np.concatenate([colour, colour[:, pick] + rng.uniform(-cdiff, cdiff, size=(colour_rows, n_pairs))], 1)
    v = rng.uniform(0, 2, size=n)
    v[pick[:zero_pairs]] = 0.0
    v[n_base:n_base + zero_pairs] = 0.0
    p = {"mean": mean, "quat": rng.normal(size=(4, n)), "log_scale": rng.uniform(np.log(0.005), np.log(0.05), (3, n)),
         "opacity_logit": rng.normal(size=n) * 2, "colour": colour}
    perm = rng.permutation(n)
    p = {k: np.ascontiguousarray(x[..., perm]).astype(np.float32) for k, x in p.items()}
    return p, v[perm].astype(np.float32)


def _dev(d):
    return {k: torch.from_numpy(np.ascontiguousarray(x)).cuda() for k, x in d.items()}


def _margins(p, nn, radius, colour_tol):
    """Relative distance of every mutual pair's two tests from their
    thresholds (FP64 of the FP32 inputs)."""
    m = p["mean"].astype(np.float64)
    ls = p["log_scale"].astype(np.float64)
    col = p["colour"].astype(np.float64).reshape(-1, m.shape[1])
    out = []
    for i, j in enumerate(nn):
        if j > i and nn[j] == i:
            d = np.linalg.norm(m[:, i] - m[:, j])
            lim = radius * min(np.exp(ls[:, i].mean()), np.exp(ls[:, j].mean()))
            cd = np.abs(col[:3, i] - col[:3, j]).max()
            out.append(min(abs(d - lim) / lim, abs(cd - colour_tol) / max(colour_tol, 1e-30)))
    return np.array(out)


def _check_nearest(p, nn_gpu):
    from scipy.spatial import cKDTree
    pts = p["mean"].astype(np.float64).T
    dist, idx = cKDTree(pts).query(pts, k=3)
    unique = dist[:, 2] - dist[:, 1] > 1e-9 * dist[:, 1]
    assert np.array_equal(nn_gpu[unique], idx[unique, 1])
    amb = np.nonzero(~unique)[0]
    for i in amb:
        d = np.linalg.norm(pts[nn_gpu[i]] - pts[i])
        assert nn_gpu[i] != i and d <= dist[i, 1] * (1 + 1e-9), i
    return idx[:, 1], int(unique.sum())


def _check_merge(p, v, nn_ref, radius, colour_tol, out_gpu, keep_gpu):
    ref, keep_ref = O.merge({k: x.astype(np.float64) for k, x in p.items()}, v.astype(np.float64), radius,
                            colour_tol, nn=nn_ref)
    n = keep_ref.size
    assert np.array_equal(keep_gpu.astype(bool), keep_ref)
    surv = np.array([i for i in range(n) if nn_ref[i] > i and nn_ref[nn_ref[i]] == i and not keep_ref[nn_ref[i]]],
                    dtype=np.int64)
    copy = np.setdiff1d(np.arange(n), surv)
    for k in PLANES:
        assert np.array_equal(out_gpu[k][..., copy], p[k][..., copy]), k
    for k in ("mean", "colour", "opacity_logit"):
        g, r = out_gpu[k][..., surv].astype(np.float64), ref[k][..., surv]
        assert np.allclose(g, r, rtol=1e-6, atol=1e-7), (k, np.abs(g - r).max())
    worst = 0.0
    for i in surv:
        S_ref = O.covariance(ref["quat"][:, i], ref["log_scale"][:, i])
        S_got = O.covariance(out_gpu["quat"][:, i].astype(np.float64), out_gpu["log_scale"][:, i].astype(np.float64))
        err = np.abs(S_got - S_ref).max() / np.abs(S_ref).max()
        worst = max(worst, err)
        assert abs(np.linalg.norm(out_gpu["quat"][:, i].astype(np.float64)) - 1.0) < 1e-6
    assert worst <= 1e-5, worst
    return surv.size, worst


@pytest.mark.parametrize("n_base,n_pairs,colour_rows", [(20000, 5000, 3), (3001, 700, 48)])
def test_merge_parity(n_base, n_pairs, colour_rows):
    radius, colour_tol = 1.0, 0.05
    say(f"[merge] n_base={n_base} n_pairs={n_pairs} colour_rows={colour_rows}")
    p, v = _cloud(n_base + colour_rows, n_base, n_pairs, colour_rows)
    n = n_base + n_pairs
    P = _dev(p)
    vd = torch.from_numpy(v).cuda()
    nn = maintain.nearest(P["mean"])
    torch.cuda.synchronize()
    nn_ref, n_unique = _check_nearest(p, nn.cpu().numpy())
    say(f"  nearest: {n_unique} of {n} unique, all valid")
    margins = _margins(p, nn_ref, radius, colour_tol)
    assert margins.size > n_pairs // 2 and margins.min() > 1e-9
    # both sides merge along the oracle's neighbours
    out, keep, _ = maintain.merge(P, vd, radius, colour_tol, nn=torch.from_numpy(nn_ref.astype(np.int32)).cuda())
    torch.cuda.synchronize()
    got = {k: x.cpu().numpy() for k, x in out.items()}
    merged, worst = _check_merge(p, v, nn_ref, radius, colour_tol, got, keep.cpu().numpy())
    assert n_pairs // 10 < merged < n_pairs
    say(f"  merged {merged} pairs, covariance error {worst:.2e}")
    # the ordered keep list and the compaction of every plane
    idx, kept = maintain.keep_list(keep)
    torch.cuda.synchronize()
    ref_idx = np.nonzero(keep.cpu().numpy())[0]
    assert int(kept.cpu()) == ref_idx.size == n - merged
    assert np.array_equal(idx.cpu().numpy()[:ref_idx.size], ref_idx)
    for k in PLANES:
        dst = maintain.compact(out[k], idx, kept)
        torch.cuda.synchronize()
        assert np.array_equal(dst.cpu().numpy()[..., :ref_idx.size], got[k][..., ref_idx]), k


def test_merge_end_to_end_with_gpu_neighbours():
    """The whole pass on GPU neighbours, on a cloud whose nearest neighbours
    are all unique: the same result as the oracle on its own."""
    p, v = _cloud(77, 8000, 2000)
    P = _dev(p)
    out, keep, nn = maintain.merge(P, torch.from_numpy(v).cuda(), 1.0, 0.05)
    torch.cuda.synchronize()
    nn_ref, n_unique = _check_nearest(p, nn.cpu().numpy())
    assert n_unique == 10000
    got = {k: x.cpu().numpy() for k, x in out.items()}
    merged, _ = _check_merge(p, v, nn_ref, 1.0, 0.05, got, keep.cpu().numpy())
    assert merged > 100


def test_merge_degenerate_cases():
    # one Gaussian: no neighbour, nothing merges, the output is a copy
    p, v = _cloud(5, 1, 0, zero_pairs=0)
    P = _dev(p)
    out, keep, nn = maintain.merge(P, torch.from_numpy(v).cuda(), 1.0, 0.05)
    torch.cuda.synchronize()
    assert nn.cpu().tolist() == [-1] and keep.cpu().tolist() == [1]
    for k in PLANES:
        assert np.array_equal(out[k].cpu().numpy(), p[k])
    # a copy of one Gaussian next to it, both invisible: equal weights, the
    # survivor is the same Gaussian
    p, v = _cloud(6, 2, 0, zero_pairs=0)
    for k in PLANES:
        p[k][..., 1] = p[k][..., 0]
    p["mean"][:, 1] += np.float32(1e-4)
    v[:] = 0.0
    out, keep, nn = maintain.merge(_dev(p), torch.from_numpy(v).cuda(), 1.0, 0.05)
    torch.cuda.synchronize()
    assert nn.cpu().tolist() == [1, 0] and keep.cpu().tolist() == [1, 0]
    got = {k: x.cpu().numpy() for k, x in out.items()}
    S0 = O.covariance(p["quat"][:, 0].astype(np.float64), p["log_scale"][:, 0].astype(np.float64))
    S1 = O.covariance(got["quat"][:, 0].astype(np.float64), got["log_scale"][:, 0].astype(np.float64))
    assert np.abs(S1 - S0).max() <= 1e-5 * np.abs(S0).max()
    assert np.allclose(got["colour"][:, 0], p["colour"][:, 0], rtol=1e-6)
    assert np.allclose(got["mean"][:, 0], p["mean"][:, 0] + np.float32(5e-5), rtol=1e-6, atol=1e-7)
    # zero radius: nothing merges
    _, keep, _ = maintain.merge(_dev(p), torch.from_numpy(v).cuda(), 0.0, 0.05)
    assert keep.cpu().tolist() == [1, 1]
    # saturated opacities (logits 40 and 45, alpha rounds to 1 in double):
    # the merged logit stays finite and equals the oracle's
    p["opacity_logit"][:] = [40.0, 45.0]
    v[:] = [1.0, 3.0]
    out, keep, _ = maintain.merge(_dev(p), torch.from_numpy(v).cuda(), 1.0, 0.05)
    torch.cuda.synchronize()
    ref, _ = O.merge(p, v, 1.0, 0.05, nn=np.array([1, 0]))
    got = float(out["opacity_logit"][0].cpu())
    assert keep.cpu().tolist() == [1, 0] and np.isfinite(got)
    assert abs(got - ref["opacity_logit"][0]) <= 1e-6 * abs(ref["opacity_logit"][0])


def test_nearest_with_a_validity_mask():
    """Invalid Gaussians are neither queried nor found: -1 for them, and the
    valid ones' neighbours are the k-d tree's over the valid set."""
    from scipy.spatial import cKDTree
    p, _ = _cloud(31, 6000, 1500)
    n = p["mean"].shape[1]
    valid = (np.random.default_rng(32).uniform(size=n) < 0.7).astype(np.int32)
    nn = maintain.nearest(torch.from_numpy(p["mean"]).cuda(), torch.from_numpy(valid).cuda())
    torch.cuda.synchronize()
    got = nn.cpu().numpy()
    idx = np.nonzero(valid)[0]
    pts = p["mean"][:, idx].astype(np.float64).T
    dist, j = cKDTree(pts).query(pts, k=3)
    unique = dist[:, 2] - dist[:, 1] > 1e-9 * dist[:, 1]
    assert np.all(got[valid == 0] == -1)
    assert np.array_equal(got[idx][unique], idx[j[unique, 1]])
    assert unique.sum() > 0.99 * idx.size
    # no valid pair at all
    one = np.zeros(n, np.int32)
    one[5] = 1
    nn = maintain.nearest(torch.from_numpy(p["mean"]).cuda(), torch.from_numpy(one).cuda())
    assert nn.cpu().numpy().tolist() == [-1] * n
