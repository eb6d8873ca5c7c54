"""Parity of the GPU mapping loss (gsr_loss_mapping through the C ABI:
(1 - lambda) L1 + lambda (1 - SSIM), the appendix's optimisation settings)
with the FP64 oracle.

Bar.  The kernel computes in FP32.  The local variance w * x^2 - mu^2 loses
about 1e-7 of w * x^2 to cancellation, which the stabiliser C2 = 9e-4 bounds
to ~1e-4 relative in SSIM's denominator, so each gradient entry is held to
1e-3 of the largest entry of its view (the 1e-3 relative gradient bar) and
the loss to 1e-6 absolute (a mean of FP32 values summed in double).  The
L1 part with lambda = 0 is exact: it equals the L1 gradient seed bit for
bit.
"""
import numpy as np
import pytest
import torch

from oracle import ssim as M

pytestmark = pytest.mark.gpu

LAM = 0.2


def say(msg):
    print(msg, flush=True)


def _cams(sizes):
    return [dict(width=w, height=h, fx=50.0, fy=50.0, cx=w / 2, cy=h / 2) for w, h in sizes]


def _images(rng, sizes, noise=0.05, equal_frac=0.02):
    xs, ys = [], []
    for w, h in sizes:
        # smooth structure plus noise, so that SSIM spans low and high variance
        u = np.linspace(0, 3, w)[None, :] + np.linspace(0, 2, h)[:, None]
        base = 0.5 + 0.3 * np.sin(u + rng.uniform(0, 6, size=(3, 1, 1)))
        x = np.clip(base + rng.normal(0, 0.1, size=(3, h, w)), 0, 1)
        y = np.clip(x + rng.normal(0, noise, size=x.shape), 0, 1)
        eq = rng.uniform(size=x.shape) < equal_frac
        y[eq] = x[eq]
        # a flat patch (zero local variance)
        x[:, : h // 3, : w // 3] = 0.4
        y[:, : h // 3, : w // 3] = 0.45
        xs.append(x.astype(np.float32))
        ys.append(y.astype(np.float32))
    return xs, ys


def _renderer(sizes):
    from paper_2601_00705_amd.render import Config, Renderer
    return Renderer(16, _cams(sizes), Config())


def _flat(arrs):
    return torch.from_numpy(np.concatenate([a.reshape(-1) for a in arrs])).cuda()


def _split(flat, sizes):
    out, o = [], 0
    for w, h in sizes:
        out.append(flat[o:o + 3 * w * h].reshape(3, h, w))
        o += 3 * w * h
    return out


def _run(R, x, y, lam):
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    dL = torch.full_like(x, np.nan)
    R.loss_mapping(x, y, lam, loss, dL)
    torch.cuda.synchronize()
    return float(loss.cpu()), dL.cpu().numpy()


def _check(got_loss, got_g, sizes, xs, ys, lam):
    ref_loss, ref_g = M.mapping_loss([a.astype(np.float64) for a in xs], [a.astype(np.float64) for a in ys], lam)
    assert abs(got_loss - ref_loss) < 1e-6, (got_loss, ref_loss)
    worst = 0.0
    for gv, rv in zip(_split(got_g, sizes), ref_g):
        scale = np.abs(rv).max()
        err = np.abs(gv - rv).max() / scale
        worst = max(worst, err)
        assert err < 1e-3, err
    say(f"  loss {got_loss:.8f} (oracle {ref_loss:.8f}); worst gradient error {worst:.2e} of the view's largest")


@pytest.mark.parametrize("sizes", [[(37, 29)], [(64, 48), (5, 3), (100, 70)], [(1, 1), (33, 1), (1, 40)]])
def test_mapping_loss_parity_ragged(sizes):
    """Tiles with ragged edges, several views of different sizes, images
    smaller than the window and one pixel wide."""
    say(f"[mapping] sizes {sizes}")
    rng = np.random.default_rng(len(sizes))
    xs, ys = _images(rng, sizes)
    R = _renderer(sizes)
    loss, g = _run(R, _flat(xs), _flat(ys), LAM)
    _check(loss, g, sizes, xs, ys, LAM)


@pytest.mark.parametrize("lam", [0.0, 1.0])
def test_mapping_loss_parity_pure_terms(lam):
    sizes = [(70, 45), (32, 32)]
    rng = np.random.default_rng(7)
    xs, ys = _images(rng, sizes)
    R = _renderer(sizes)
    loss, g = _run(R, _flat(xs), _flat(ys), lam)
    _check(loss, g, sizes, xs, ys, lam)


def test_lambda_zero_equals_the_l1_seed_and_identical_images_give_zero():
    sizes = [(50, 41), (16, 9)]
    rng = np.random.default_rng(8)
    xs, ys = _images(rng, sizes)
    R = _renderer(sizes)
    x, y = _flat(xs), _flat(ys)
    _, g = _run(R, x, y, 0.0)
    dl1 = torch.empty_like(x)
    R.loss_l1(x, y, dl1)
    torch.cuda.synchronize()
    assert np.array_equal(g, dl1.cpu().numpy())
    loss, g = _run(R, x, x, 1.0)
    # SSIM = 1 is a maximum: the gradient vanishes up to FP32 cancellation
    # (entries of order 1e2 / (3 P) when the images differ)
    assert abs(loss) < 1e-6 and np.abs(g).max() * 3 * sum(w * h for w, h in sizes) < 1e-2


def test_l1_seed_matches_the_oracle():
    """The L1 seed of the step (gsr_loss_l1, dL/dC = sign(C - target) /
    (3 pixels), sign(0) = 0) against the oracle's lambda = 0 mapping-loss
    gradient, on three views with 2 % of the entries exactly equal: the signs
    agree exactly (the float32 difference of two floats has the sign of the
    exact one, and is zero only when they are equal), the magnitudes to the
    rounding of 1 / (3 pixels) to float32."""
    sizes = [(64, 48), (37, 29), (1, 9)]
    rng = np.random.default_rng(10)
    xs, ys = _images(rng, sizes)
    R = _renderer(sizes)
    x, y = _flat(xs), _flat(ys)
    g = torch.full_like(x, np.nan)
    R.loss_l1(x, y, g)
    torch.cuda.synchronize()
    _, ref = M.mapping_loss([a.astype(np.float64) for a in xs], [a.astype(np.float64) for a in ys], 0.0)
    ref = np.concatenate([r.reshape(-1) for r in ref])
    got = g.cpu().numpy().astype(np.float64)
    assert np.array_equal(np.sign(got), np.sign(ref))
    assert (ref == 0).mean() > 0.01
    np.testing.assert_allclose(got, ref, rtol=2.0 ** -23, atol=0)


def test_mapping_loss_deterministic():
    sizes = [(130, 90), (64, 64)]
    rng = np.random.default_rng(9)
    xs, ys = _images(rng, sizes)
    R = _renderer(sizes)
    x, y = _flat(xs), _flat(ys)
    a = _run(R, x, y, LAM)
    b = _run(R, x, y, LAM)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


def test_mapping_loss_full_window_sampled():
    """The ten-view window's resolutions (4 x 640x480, 4 x 1200x680,
    2 x 320x240): the loss against the oracle over every pixel, the gradient
    at 300 sampled pixels from crops (a gradient entry depends on the images
    within 10 pixels only; a crop of radius 20 clipped to the image gives the
    oracle the same value)."""
    sizes = [(640, 480)] * 4 + [(1200, 680)] * 4 + [(320, 240)] * 2
    say("[mapping] full window: 10 views")
    rng = np.random.default_rng(10)
    xs, ys = _images(rng, sizes)
    R = _renderer(sizes)
    loss, g = _run(R, _flat(xs), _flat(ys), LAM)
    gs = _split(g, sizes)
    n = 3.0 * sum(w * h for w, h in sizes)
    l1 = sum(np.abs(x.astype(np.float64) - y).sum() for x, y in zip(xs, ys))
    ssum = 0.0
    for x, y in zip(xs, ys):
        for c in range(3):
            ssum += M.ssim_map(x[c], y[c])[0].sum()
    ref_loss = (1 - LAM) * l1 / n + LAM * (1 - ssum / n)
    say(f"  loss {loss:.8f} (oracle {ref_loss:.8f})")
    assert abs(loss - ref_loss) < 1e-6
    samples = []
    for k in range(300):
        v = int(rng.integers(len(sizes)))
        w, h = sizes[v]
        # border pixels are over-sampled
        qx = int(rng.integers(w)) if k % 3 else int(rng.choice([0, 1, 4, w - 5, w - 2, w - 1]))
        qy = int(rng.integers(h)) if k % 5 else int(rng.choice([0, 3, h - 4, h - 1]))
        c = int(rng.integers(3))
        x0, y0 = max(0, qx - 20), max(0, qy - 20)
        cx = xs[v][c, y0:qy + 21, x0:qx + 21].astype(np.float64)
        cy = ys[v][c, y0:qy + 21, x0:qx + 21].astype(np.float64)
        ref = (1 - LAM) * np.sign(cx - cy) / n - LAM / n * M.ssim_grad(cx, cy, np.ones_like(cx))
        samples.append((v, c, qx, qy, ref[qy - y0, qx - x0]))
    scale = max(abs(r) for *_, r in samples)
    worst = 0.0
    for v, c, qx, qy, r in samples:
        err = abs(gs[v][c, qy, qx] - r) / scale
        worst = max(worst, err)
        assert err < 1e-3, (v, c, qx, qy, gs[v][c, qy, qx], r)
    say(f"  worst sampled gradient error {worst:.2e} of the largest sampled entry")
