"""Parity of the GPU map maintenance (gsr_adam_step, gsr_covis, gsr_prune,
gsr_compact through the C ABI) with the FP64 oracle.

Bar.  Adam: each step starts both sides from the GPU's FP32 state; the new
parameters agree within 4 ulp of the parameter plus 1e-5 of the step's
learning rate (the FP32 update lr m / (sqrt(v) + eps) is good to a few
ulp), v within 1e-5 relative, m within 1e-5 relative plus 1e-6 of the
plane's largest |m| (b1 m + (1 - b1) g can cancel), the gradient norm
within 1e-12 relative (both sum in double).  Co-visibility: counts exact (integer) and
the IoU equal (the same double division).  Pruning: the decisions are
taken in double on both sides, so the kept lists are equal, except for a
Gaussian whose trace or opacity lies within 1e-12 of its threshold (none
occur here); compaction is a gather, exact.
"""
import numpy as np
import pytest
import torch

from oracle import optim as O

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2601_00705_amd import maintain


def say(msg):
    print(msg, flush=True)


def _planes(rng, n, colour_rows, scale=1.0):
    shapes = {"mean": (3, n), "quat": (4, n), "log_scale": (3, n), "opacity_logit": (n,),
              "colour": (colour_rows, n)}
    return {k: (rng.normal(size=s) * scale).astype(np.float32) for k, s in shapes.items()}


def _dev(d):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in d.items()}


def _host(d):
    return {k: v.cpu().numpy().astype(np.float64) for k, v in d.items()}


@pytest.mark.parametrize("n,colour_rows", [(4096, 3), (10007, 3), (999, 48)])
def test_adam_parity(n, colour_rows):
    """Three steps (clipping active in the first two, not in the third), the
    vectorised path (n a multiple of 4) and the scalar one, SH colour."""
    say(f"[adam] n={n} colour_rows={colour_rows}")
    rng = np.random.default_rng(n)
    params = _dev(_planes(rng, n, colour_rows))
    opt = maintain.Adam(params, ema=0.1)
    for t, gscale in enumerate((1.0, 0.1, 1e-4), start=1):
        grads = _dev(_planes(rng, n, colour_rows, gscale))
        before = (_host(params), _host(opt.m), _host(opt.v), opt.anchor.cpu().numpy().astype(np.float64))
        opt.step(params, grads)
        torch.cuda.synchronize()
        ref_p, ref_m, ref_v, ref_a, ref_norm = O.adam_step(before[0], _host(grads), before[1], before[2], before[3],
                                                           opt.lr, t, max_norm=1.0, ema=0.1)
        assert abs(float(opt.norm.cpu()) - ref_norm) <= 1e-12 * ref_norm
        for k in O.PLANES:
            got = params[k].cpu().numpy().astype(np.float64)
            tol = 4 * np.spacing(np.abs(ref_p[k]).astype(np.float32)).astype(np.float64) + 1e-5 * opt.lr[k]
            assert np.all(np.abs(got - ref_p[k]) <= tol), (t, k, np.abs(got - ref_p[k]).max())
            # m = b1 m + (1 - b1) g can cancel: FP32 keeps it to ~1e-7 of the terms
            assert np.allclose(opt.m[k].cpu().numpy(), ref_m[k], rtol=1e-5, atol=1e-6 * np.abs(ref_m[k]).max()), \
                (t, k)
            assert np.allclose(opt.v[k].cpu().numpy(), ref_v[k], rtol=1e-5, atol=1e-30), (t, k)
        tol = 4 * np.spacing(np.abs(ref_a).astype(np.float32)).astype(np.float64) + 1e-5 * opt.lr["mean"]
        assert np.all(np.abs(opt.anchor.cpu().numpy() - ref_a) <= tol)
        say(f"  step {t}: norm {ref_norm:.4g}")


def test_adam_window_size():
    """The mapping window's Gaussian count (1M, RGB), one step."""
    n = 1_000_000
    rng = np.random.default_rng(5)
    params = _dev(_planes(rng, n, 3))
    opt = maintain.Adam(params, ema=0.05)
    grads = _dev(_planes(rng, n, 3, 1e-3))
    before = _host(params)
    a0 = opt.anchor.cpu().numpy().astype(np.float64)
    opt.step(params, grads)
    torch.cuda.synchronize()
    z = {k: np.zeros_like(v) for k, v in before.items()}
    ref_p, _, _, ref_a, ref_norm = O.adam_step(before, _host(grads), z, z, a0, opt.lr, 1, ema=0.05)
    assert abs(float(opt.norm.cpu()) - ref_norm) <= 1e-12 * ref_norm
    for k in O.PLANES:
        got = params[k].cpu().numpy().astype(np.float64)
        tol = 4 * np.spacing(np.abs(ref_p[k]).astype(np.float32)).astype(np.float64) + 1e-5 * opt.lr[k]
        assert np.all(np.abs(got - ref_p[k]) <= tol), k


def test_covis_parity():
    rng = np.random.default_rng(6)
    P = 640 * 480 + 3
    key = rng.uniform(size=P).astype(np.float32)
    frames = rng.uniform(size=(6, P)).astype(np.float32)
    frames[1] = key
    frames[2] = 1.0
    frames[3] = 0.0
    frames[4, ::2] = key[::2]
    for tau in (0.02, 0.5):
        counts, iou = maintain.covis(torch.from_numpy(key).cuda(), torch.from_numpy(frames).cuda(), tau)
        torch.cuda.synchronize()
        ref = O.covis(key, frames, tau)
        c = counts.cpu().numpy()
        io = iou.cpu().numpy()
        for f, (inter, uni, r) in enumerate(ref):
            assert (c[f, 0], c[f, 1]) == (inter, uni), (tau, f)
            assert io[f] == r, (tau, f)
    # nothing visible anywhere
    counts, iou = maintain.covis(torch.ones(100, device="cuda"), torch.ones(2, 100, device="cuda"), 0.1)
    assert counts.cpu().numpy().tolist() == [[0, 0], [0, 0]] and iou.cpu().numpy().tolist() == [0.0, 0.0]


def _prune_case(rng, n, m_min=2, v_min=0.3, sigma_max=1.5, alpha_min=0.05):
    m_obs = rng.integers(0, 6, size=n).astype(np.int32)
    v_vis = rng.uniform(0, 2, size=n).astype(np.float32)
    ls = rng.uniform(-3, 0.5, size=(3, n)).astype(np.float32)
    op = (rng.normal(size=n) * 3).astype(np.float32)
    d = _dev({"m": m_obs, "v": v_vis, "ls": ls, "op": op})
    keep, kept = maintain.prune(d["m"], d["v"], d["ls"], d["op"], m_min, v_min, sigma_max, alpha_min)
    torch.cuda.synchronize()
    ref = np.nonzero(O.prune_keep(m_obs, v_vis.astype(np.float64), ls.astype(np.float64), op.astype(np.float64),
                                  m_min, np.float64(np.float32(v_min)), np.float64(np.float32(sigma_max)),
                                  np.float64(np.float32(alpha_min))))[0]
    k = int(kept.cpu())
    assert k == ref.size
    assert np.array_equal(keep.cpu().numpy()[:k], ref)
    return keep, kept, ls, ref


def test_prune_and_compact_parity():
    rng = np.random.default_rng(7)
    for n in (1, 2047, 2048, 100_003):
        keep, kept, ls, ref = _prune_case(rng, n)
        if ref.size:
            src = torch.from_numpy(ls).cuda()
            dst = maintain.compact(src, keep, kept)
            torch.cuda.synchronize()
            assert np.array_equal(dst.cpu().numpy()[:, :ref.size], ls[:, ref])
    # everything dropped, everything kept
    _, kept, _, ref = _prune_case(rng, 5000, m_min=10)
    assert int(kept.cpu()) == 0
    _, kept, _, ref = _prune_case(rng, 5000, m_min=0, v_min=-1.0, sigma_max=1e6, alpha_min=0.0)
    assert int(kept.cpu()) == 5000
