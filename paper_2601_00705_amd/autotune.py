"""Tile-shape and LDS-batch autotuner.

For a workload shape (the multiset of view resolutions, the Gaussian count
rounded up to a power of two, the SH degree, the GPU architecture) it times
whole fwd+bwd steps (projection, binning, compositing forward, L1 seed,
compositing backward, projection backward) for every candidate
(tile_w, tile_h, batch) with HIP events and keeps the fastest.  Results are
cached as JSON: a cache committed beside this module (measured on MI355X)
is read first, then the user cache (GSR_AUTOTUNE_CACHE or
~/.cache/gsr/autotune.json), which tune() also writes.
"""
from __future__ import annotations

import json
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
SHIPPED_CACHE = os.path.join(HERE, "autotune_cache.json")
CANDIDATES = [(8, 8, 128), (16, 8, 128), (8, 16, 128), (16, 16, 64), (16, 16, 128), (16, 16, 256),
              (32, 8, 128), (32, 16, 64), (32, 16, 128), (16, 32, 128)]


def _user_cache_path():
    return os.environ.get("GSR_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "gsr", "autotune.json"))


def shape_key(cams, n, sh_degree, arch="gfx950"):
    views = {}
    for c in cams:
        k = f"{int(c['width'])}x{int(c['height'])}"
        views[k] = views.get(k, 0) + 1
    vs = ",".join(f"{k}*{views[k]}" for k in sorted(views))
    nb = 1 << max(0, int(n) - 1).bit_length()
    return f"{arch}|{vs}|n<={nb}|sh{sh_degree}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(cams, n, sh_degree, arch="gfx950"):
    """(tile_w, tile_h, batch) from the caches, or None."""
    key = shape_key(cams, n, sh_degree, arch)
    for path in (_user_cache_path(), SHIPPED_CACHE):
        ent = _load(path).get(key)
        if ent:
            return tuple(ent["best"])
    return None


def tune(params, cams, poses, target, sh_degree, pose_only=None, candidates=CANDIDATES, steps=5,
         warmup=2, arch="gfx950", log=None):
    """Times each candidate on the given (device-resident) workload and
    returns {"best": (tw, th, batch), "ms": {candidate: median ms}}."""
    import torch
    from .render import Config, Renderer
    n = int(params["opacity_logit"].shape[0])
    P = sum(int(c["width"]) * int(c["height"]) for c in cams)
    results = {}
    for (tw, th, batch) in candidates:
        cfg = Config(tile_w=tw, tile_h=th, batch=batch, sh_degree=sh_degree)
        R = Renderer(n, cams, cfg)
        R.project(params, poses)
        R.bin()
        need, _ = R.pair_count()
        R._make(int(need * 1.15) + 4096)
        rgb = torch.empty(3 * P, device=poses.device)
        T = torch.empty(P, device=poses.device)
        nc = torch.empty(P, dtype=torch.int32, device=poses.device)
        dL = torch.empty(3 * P, device=poses.device)
        grads = {k: torch.empty_like(v) for k, v in params.items()}
        d_xi = torch.empty(len(cams), 6, device=poses.device)

        def step():
            R.project(params, poses)
            R.bin()
            R.render_fwd(rgb, T, nc)
            R.loss_l1(rgb, target, dL)
            R.raster_bwd(T, nc, dL)
            R.project_bwd(params, poses, pose_only, grads, d_xi)

        times = []
        for it in range(warmup + steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            step()
            e1.record()
            torch.cuda.synchronize()
            if it >= warmup:
                times.append(e0.elapsed_time(e1))
        results[f"{tw}x{th}/{batch}"] = statistics.median(times)
        if log:
            log(f"autotune {tw}x{th} batch {batch}: {results[f'{tw}x{th}/{batch}']:.3f} ms")
        del R
    best_name = min(results, key=results.get)
    t, b = best_name.split("/")
    best = (int(t.split("x")[0]), int(t.split("x")[1]), int(b))
    key = shape_key(cams, n, sh_degree, arch)
    path = _user_cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        cache = _load(path)
        cache[key] = {"best": list(best), "ms": results}
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    except OSError:
        pass
    return {"best": best, "ms": results, "key": key}
