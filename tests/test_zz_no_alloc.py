"""The no-allocation pruning entry point (gsr_prune_noalloc, through the C
ABI) against gsr_prune with a caller workspace: identical kept lists and
counts, bit for bit, on two calls in a row, the second smaller than the
first (the fixed scratch still holds the first call's counts beyond the
second's blocks)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    dev = "cuda"
    m_obs = torch.from_numpy(rng.integers(0, 6, n).astype(np.int32)).to(dev)
    v_vis = torch.from_numpy(rng.uniform(0, 2, n).astype(np.float32)).to(dev)
    log_scale = torch.from_numpy(rng.uniform(np.log(0.01), np.log(2.0), (3, n)).astype(np.float32)).to(dev)
    logit = torch.from_numpy(rng.normal(0, 2, n).astype(np.float32)).to(dev)
    return m_obs, v_vis, log_scale, logit


def _both(n, seed):
    from paper_2601_00705_amd import lib
    m_obs, v_vis, ls, logit = _inputs(n, seed)
    cfg = lib.PruneConfig(2, 0.3, 1.5, 0.05)
    stream = torch.cuda.current_stream().cuda_stream
    keep_a = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    kept_a = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    ws = torch.empty(max(lib.gsr_prune_workspace_bytes(n), 4), dtype=torch.uint8, device="cuda")
    keep_b = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    kept_b = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    print(f"[no-alloc] gsr_prune n={n}", flush=True)
    lib.gsr_prune(n, m_obs, v_vis, ls, logit, cfg, keep_a, kept_a, ws, stream)
    torch.cuda.synchronize()
    print(f"[no-alloc] gsr_prune_noalloc n={n}", flush=True)
    lib.gsr_prune_noalloc(n, m_obs, v_vis, ls, logit, cfg, keep_b, kept_b, stream)
    torch.cuda.synchronize()
    ka, kb = int(kept_a.cpu()), int(kept_b.cpu())
    return ka, kb, keep_a.cpu().numpy(), keep_b.cpu().numpy()


def test_prune_noalloc_matches_prune_on_two_calls():
    for n, seed in ((1_000_003, 1), (70_001, 2)):
        ka, kb, a, b = _both(n, seed)
        assert 0 < ka < n and ka == kb, (n, ka, kb)
        assert np.array_equal(a[:ka], b[:kb]), n
        assert np.all(np.diff(b[:kb]) > 0)
