#!/usr/bin/env python
"""Throughput of the differentiable Gaussian-splatting renderer on one MI355X.

A step is one pass of the whole path over one batch of views: projection,
binning (pair emission + LDS radix sort + tile ranges), compositing forward,
the L1 photometric gradient seed, compositing backward and projection
backward (all parameters and the pose twists).  Inputs are synthetic and
seeded (paper_2601_00705_amd.scenes) and resident in HBM before timing.

The map is stored in the library's spatial order (gsr_spatial_order, as
the map maintenance keeps it; the reorder runs once, outside the timed
region, and is timed with the maintenance); a comparison leg times the same
step on the generator's order.

Batched mode: all views of the workload in one plan, the step captured once
in a HIP graph (torch.cuda.CUDAGraph over the library's stream) and
replayed.  Plain mode: one plan per view, launched view after view on one
stream without a graph.  Prints one JSON line on stdout; details on stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X peaks (published): HBM 8 TB/s; FP32 vector 157.3 TFLOP/s (256 CUs x
# 2.4 GHz x 256 flops per clock and CU, an FMA counted as two flops, packed).
# The VALU issue model (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12
# lane-instructions/s unpacked, a transcendental taking 4 issue slots) serves
# the mapping loss only: the compositing backward issues faster than it (some
# instructions take fewer than four cycles), so its roofline is the FP32
# peak.
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
VALU_PEAK_TSLOTS = 256 * 4 * 16 * 2.4e9 / 1e12

# Algorithmic work per evaluation (one pixel against one list entry, up to the
# pixel's last contributor) of the compositing kernels, as the per-pixel
# formulas of Eq. (alpha) and its backward count it: forward about 18 FP32
# operations and one exponential, backward about 55 operations, one
# exponential and one reciprocal.  These are the roofline's counts, each
# operation taken as one flop against the FP32 vector peak.
OPS_FWD_PER_EVAL = 18 + 1
OPS_BWD_PER_EVAL = 55 + 1 + 1
# Algorithmic work of the other stages per unit (HBM bytes; FP32 operations
# where they matter), for the step-level roofline:
#   projection: read 56 B per Gaussian (236 B with SH degree 3), write a
#     52-byte record per live (Gaussian, view) slot, ~124 operations per slot
#     (~100 more with SH degree 3)
#   binning: 8 B per live slot (the scan), 12 B per pair emitted, one read and
#     write of each pair by the sort (24 B), 8 B per pair for the tile ranges
#   compositing: a 40-byte record gathered per pair; 20 B per pixel written
#     (forward) or read (backward)
#   L1 seed: render and target read, gradient written, 36 B per pixel
#   projection backward: parameters read and gradients written per Gaussian
#     (56 + 56 B, 236 + 236 B with SH degree 3), 36 B of screen-space gradient
#     read per live slot, ~250 operations per live slot
BYTES_PROJ_PER_GAUSSIAN = {False: 56, True: 236}
BYTES_PROJ_PER_SLOT = 52
OPS_PROJ_PER_SLOT = {False: 124, True: 224}
BYTES_BIN_PER_SLOT = 8
BYTES_BIN_PER_PAIR = 12 + 24 + 8
BYTES_RASTER_PER_PAIR = 40
BYTES_RASTER_PER_PIXEL = 20
BYTES_LOSS_PER_PIXEL = 36
BYTES_PBWD_PER_GAUSSIAN = {False: 112, True: 472}
BYTES_PBWD_PER_SLOT_READ = 36
OPS_PBWD_PER_SLOT = 250
# Tracking loss: weight thresholds (the paper gives none; accumulated opacity
# saturates the weight from 0.5, an observed gradient norm from 0.05 per
# pixel), and its algorithmic HBM bytes per pixel over its three passes: the
# exposure sums read render and observation (24 B); the sign sums read them
# and T_final (28 B); the gradient reads the same and writes dL/drgb and
# dL/dT_final (28 + 16 B)
TRACK_TAU_ALPHA = 0.5
TRACK_TAU_GRAD = 0.05
BYTES_TRACK_PER_PIXEL = 24 + 28 + 28 + 16
# Mapping loss (L1 + lambda D-SSIM, lambda_dssim = 0.2 in the appendix's
# optimisation settings): algorithmic VALU issue slots per pixel and channel
# of the separable filtering without aprons: the five products along rows
# (11 taps x 7 operations), along columns (11 x 5 FMA), SSIM and its three
# partials (~50, two divisions at ~12 slots each), the partials along rows
# (11 x 3 FMA) and columns (11 x 3 FMA) and the gradient (5); its
# algorithmic HBM bytes per pixel: render and target read, gradient written
MAP_LAMBDA = 0.2
SLOTS_MAP_PER_PIXEL = 3 * (77 + 55 + 50 + 33 + 38)
BYTES_MAP_PER_PIXEL = 12 + 12 + 12
# Seeding: FP64 peak of the vector units (published), and the FP64 operations
# per reference pixel and neighbour: the 4x4 system (16), six sweeps of the
# one-sided Jacobi SVD (6 rotations x 87: three 4-term dot products, the
# rotation, both columns of A and V), the singular vector choice (32), the
# two reprojections, the error and the baseline angle (~80)
FP64_PEAK_TFLOPS = 78.6
FLOPS_SEED_PER_HYPOTHESIS = 16 + 6 * 6 * 87 + 32 + 80

# files whose text defines the compositing kernels (a counter summary is only
# used while they are unchanged)
KERNEL_SOURCES = ("paper_2601_00705_amd/csrc/raster.hip", "paper_2601_00705_amd/csrc/gsr_device.h",
                  "paper_2601_00705_amd/csrc/kernels.h")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3, help="workload index 0..4")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-views", type=str, default=None, help="comma list of views for the oracle sample")
    ap.add_argument("--tile", type=str, default=None, help="WxH[/batch] (default: autotuned)")
    ap.add_argument("--autotune", action="store_true", help="re-run the tile/batch autotuner")
    ap.add_argument("--copy-probe", action="store_true", help="run a plain device copy of known size first")
    ap.add_argument("--no-seeding", action="store_true", help="skip the seeding measurement")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the loss and map-maintenance measurements (short profiler runs)")
    ap.add_argument("--no-mixed", action="store_true", help="skip timing the mixed-precision variant")
    ap.add_argument("--precision", choices=("fp32", "mixed"), default="fp32",
                    help="precision of the headline step (default fp32)")
    ap.add_argument("--no-second", action="store_true",
                    help="skip the second leg (the 3M-Gaussian tracking-and-mapping batch)")
    ap.add_argument("--deterministic", action="store_true",
                    help="bitwise-reproducible backward (fixed-point accumulation)")
    ap.add_argument("--loss", choices=("l1", "track", "mapping"), default="l1",
                    help="gradient seed of the step: L1 (default), the tracking loss or the mapping loss")
    ap.add_argument("--map-order", choices=("spatial", "given"), default="spatial",
                    help="storage order of the map: the library's spatial order (default) or the generator's")
    ap.add_argument("--brick", type=int, default=None,
                    help="Gaussians per brick of the spatial order (default: the library's)")
    ap.add_argument("--no-given", action="store_true",
                    help="skip the comparison leg on the generator's order")
    return ap.parse_args()


def target_images(w, params_d, poses_d, cfg, Renderer, torch):
    """Target images of the workload, rendered once on the GPU (untimed) or
    taken from the workload's own images."""
    import numpy as np
    cams = w["cams"]
    if "targets" in w:
        return torch.from_numpy(np.concatenate([t.reshape(-1) for t in w["targets"]])).cuda()
    R = Renderer(w["params"]["opacity_logit"].shape[0], cams, cfg)
    if "target_params" in w:
        P = {k: torch.from_numpy(v).cuda() for k, v in w["target_params"].items()}
        rgb, _, _, _ = R.forward_all(P, poses_d)
    else:
        tp = torch.from_numpy(w["target_poses"].astype(np.float32)).cuda()
        rgb, _, _, _ = R.forward_all(params_d, tp)
    torch.cuda.synchronize()
    out = rgb.clone()
    del R
    return out


class Step:
    """Buffers and the C-ABI call sequence of one step for one plan."""

    def __init__(self, R, params, poses, target, pose_only, torch, loss="l1"):
        self.R, self.params, self.poses, self.target, self.pose_only = R, params, poses, target, pose_only
        self.loss = loss
        P = R.total_pixels
        dev = poses.device
        self.rgb = torch.empty(3 * P, dtype=R.image_dtype, device=dev)
        self.T = torch.empty(P, device=dev)
        self.nc = torch.empty(P, dtype=torch.int32, device=dev)
        self.dL = torch.empty(3 * P, device=dev)
        self.dT = torch.empty(P, device=dev)
        self.loss_v = torch.empty(len(R.cams), dtype=torch.float64, device=dev)
        self.loss_m = torch.empty(1, dtype=torch.float64, device=dev)
        self.expo = torch.empty(len(R.cams), 2, dtype=torch.float64, device=dev)
        self.grads = {k: torch.empty_like(v) for k, v in params.items()}
        self.d_xi = torch.empty(len(R.cams), 6, device=dev)

    def stages(self):
        R = self.R
        return [
            ("project", lambda: R.project(self.params, self.poses)),
            ("bin", lambda: R.bin()),
            ("raster_fwd", lambda: R.render_fwd(self.rgb, self.T, self.nc)),
            ("loss", self.seed),
            ("raster_bwd", lambda: R.raster_bwd(self.T, self.nc, self.dL, self.dT if self.loss == "track" else None)),
            ("project_bwd", lambda: R.project_bwd(self.params, self.poses, self.pose_only, self.grads, self.d_xi)),
        ]

    def seed(self):
        if self.loss == "track":
            self.track()
        elif self.loss == "mapping":
            self.mapping()
        else:
            self.R.loss_l1(self.rgb, self.target, self.dL)

    def track(self):
        self.R.loss_track(self.rgb, self.T, self.target, TRACK_TAU_ALPHA, TRACK_TAU_GRAD, self.loss_v, self.expo,
                          self.dL, self.dT)

    def mapping(self):
        self.R.loss_mapping(self.rgb, self.target, MAP_LAMBDA, self.loss_m, self.dL)

    def run(self):
        for _, f in self.stages():
            f()


def sized_renderer(Renderer, n, cams, cfg, params, poses, torch, slack=1.15):
    R = Renderer(n, cams, cfg)
    R.project(params, poses)
    R.bin()
    need, _ = R.pair_count()
    R._make(int(need * slack) + 4096)
    return R, need


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, cfg):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary (profiles/<kernel>.<workload>.md), or None when there is none
    for this workload and tile setting or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"{kernel}.{workload}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            k, sep, v = line.strip().lstrip("-* ").partition(":")
            if sep:
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("sources_sha256") != sources_digest():
        return None
    if fields.get("tile") != f"{cfg.tile_w}x{cfg.tile_h}/{cfg.batch}":
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _graph_ms(torch, fn, reps, calls=20):
    """Average device time of fn() replayed from a graph of `calls` calls."""
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        fn()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            for _ in range(calls):
                fn()
    torch.cuda.synchronize()
    g.replay()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / (calls * reps)


def maintenance_measurement(torch, w, params, T_final, cams, reps, log):
    """Map maintenance at the workload's size: one optimiser step over every
    Gaussian parameter (with the anchor), the co-visibility of every view
    against the first one of its size, and pruning with the compaction of
    the log-scales.  All bound by HBM traffic; bytes per unit:
      Adam: per float, read p, g, m, v and write p, m, v (28 B), plus the
            norm pass reading g (4 B); per mean float the anchor (8 B);
      co-visibility: per frame pixel, T of the frame and of the key (8 B);
      pruning: per Gaussian, two passes reading m, v, three log-scales and
            the opacity logit (2 x 24 B), the kept index (4 B), and the
            compaction of 3 log-scale rows (read + write 24 B);
      merging: per Gaussian, read its neighbour index, the neighbour's
            index, its visibility and every parameter row, write every row
            and the keep flag (8 + 4 + 2 x 4 x rows + 4 B), then the keep
            list (two passes over the flags, 8 B, and the index, 4 B);
      spatial reorder: per Gaussian, the means twice (24 B), the codes and
            indices written (8 B), four radix passes each reading them twice
            and writing them once (4 x 24 B), the brick gather (8 B), then
            every row gathered (12 B per row: index, read, write).
    The nearest-neighbour search before merging is a grid search, reported
    by its time only."""
    import numpy as np
    from paper_2601_00705_amd import maintain
    n = int(params["opacity_logit"].shape[0])
    P = {k: v.clone() for k, v in params.items()}
    G = {k: torch.randn_like(v) * 1e-3 for k, v in P.items()}
    opt = maintain.Adam(P, ema=0.05)
    floats = sum(v.numel() for v in P.values())
    t_adam = _graph_ms(torch, lambda: opt.step(P, G), reps)
    b_adam = 32 * floats + 8 * P["mean"].numel()
    # co-visibility: views of the key's size
    sizes = [(c["width"], c["height"]) for c in cams]
    key = sizes[0]
    idx = [v for v, s in enumerate(sizes) if s == key]
    offs = np.cumsum([0] + [wd * ht for wd, ht in sizes])
    frames = torch.stack([T_final[offs[v]:offs[v + 1]] for v in idx]).contiguous()
    t_cov = _graph_ms(torch, lambda: maintain.covis(frames[0], frames, 0.05), reps)
    b_cov = 8 * frames.numel()
    m_obs = torch.randint(0, 6, (n,), dtype=torch.int32, device=P["mean"].device)
    v_vis = torch.rand(n, device=P["mean"].device) * 2
    state = {}

    def prune_and_compact():
        keep, kept = maintain.prune(m_obs, v_vis, P["log_scale"], P["opacity_logit"], 2, 0.3, 1.5, 0.05)
        state["ls"] = maintain.compact(P["log_scale"], keep, kept)

    t_pr = _graph_ms(torch, prune_and_compact, reps)
    b_pr = (2 * 24 + 4 + 24) * n
    t_nn = _graph_ms(torch, lambda: maintain.nearest(P["mean"]), max(reps // 4, 2), calls=2)
    nn = maintain.nearest(P["mean"])

    def merge_and_list():
        _, keep, _ = maintain.merge(P, v_vis, 1.0, 0.05, nn=nn)
        state["list"] = maintain.keep_list(keep)

    t_mg = _graph_ms(torch, merge_and_list, reps)
    rows = floats // n
    b_mg = (8 + 4 + 8 * rows + 4 + 8 + 4) * n

    def reorder():
        state["ord"] = maintain.permute(P, maintain.spatial_order(P["mean"]))

    t_or = _graph_ms(torch, reorder, max(reps // 4, 2), calls=2)
    b_or = (128 + 12 * rows) * n
    out = {"nearest": {"ms": t_nn, "work": f"{n} Gaussians"}}
    log(f"maintenance nearest: {t_nn:.4f} ms")
    for name, t, b, unit in (("adam", t_adam, b_adam, f"{floats} floats"),
                             ("covis", t_cov, b_cov, f"{len(idx)} frames x {key[0]}x{key[1]}"),
                             ("prune_compact", t_pr, b_pr, f"{n} Gaussians"),
                             ("merge_list", t_mg, b_mg, f"{n} Gaussians, {rows} rows"),
                             ("spatial_reorder", t_or, b_or, f"{n} Gaussians, {rows} rows")):
        out[name] = {"ms": t, "bound": "hbm", "achieved": b / (t * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, "work": unit}
        log(f"maintenance {name}: {t:.4f} ms, {out[name]['achieved']:.0f} GB/s ({out[name]['frac']:.2f} of HBM)")
    return out


def seeding_measurement(torch, reps, log):
    """Seeding at the mapping workload's shape: 500,000 reference pixels of a
    1200x680 keyframe with 4 neighbours (synthetic correspondences of the
    analytic room, 10 % outliers), then the nearest-neighbour scale."""
    from paper_2601_00705_amd import scenes, seeding
    d = scenes.seed_inputs(2601, 500_000, width=1200, height=680, f=600.0)
    views = [dict(P=d["Ps"][v], centre=d["centres"][v], width=d["cams"][v]["width"],
                  height=d["cams"][v]["height"], image=torch.from_numpy(d["images"][v]).cuda(),
                  gain=d["expo"][v, 0], bias=d["expo"][v, 1]) for v in range(len(d["images"]))]
    cfg = dict(max_reproj=2.0, min_parallax=0.5 * 3.141592653589793 / 180.0, alpha_lo=0.05, alpha_hi=0.95)
    dev = {k: torch.from_numpy(d[k]).cuda() for k in ("xr", "xn", "kappa")}
    n, K = d["xr"].shape[1], d["xn"].shape[0]
    sc = seeding.Scaler(n)
    out = seeding.triangulate(views, cfg, dev["xr"], dev["xn"], dev["kappa"], diagnostics=False)
    ls = sc(out["mean"], out["valid"])
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_tri = t_knn = 0.0
    for _ in range(reps):
        ev[0].record()
        seeding.triangulate(views, cfg, dev["xr"], dev["xn"], dev["kappa"], diagnostics=False)
        ev[1].record()
        sc(out["mean"], out["valid"], log_scale=ls)
        ev[2].record()
        torch.cuda.synchronize()
        t_tri += ev[0].elapsed_time(ev[1])
        t_knn += ev[1].elapsed_time(ev[2])
    t_tri /= reps
    t_knn /= reps
    # the anisotropic initialisation (plane fit within 1 cm, about 60 seeds)
    diag = seeding.triangulate(views, cfg, dev["xr"], dev["xn"], dev["kappa"], diagnostics=True)
    fr = dict(P_ref=d["Ps"][0].reshape(-1), centre_ref=d["centres"][0], radius=0.01)
    quat, fls = sc.frame(diag["mean"], diag["valid"], diag["err"], diag["angle"], **fr)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        sc.frame(diag["mean"], diag["valid"], diag["err"], diag["angle"], quat=quat, log_scale=fls, **fr)
    ev[1].record()
    torch.cuda.synchronize()
    t_frame = ev[0].elapsed_time(ev[1]) / reps
    flops = FLOPS_SEED_PER_HYPOTHESIS * K * n
    res = {"points": n, "neighbours": K, "kept": int(out["valid"].sum()), "triangulate_ms": t_tri,
           "scale_ms": t_knn, "frame_ms": t_frame, "frame_radius": fr["radius"],
           "points_per_s": n / ((t_tri + t_knn) * 1e-3),
           "roofline": {"bound": "alu", "kernel": "seed_triangulate",
                        "achieved": flops / (t_tri * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
                        "unit": "TFLOP/s (FP64)", "work": f"{FLOPS_SEED_PER_HYPOTHESIS} x {K} x {n}"}}
    res["roofline"]["frac"] = res["roofline"]["achieved"] / FP64_PEAK_TFLOPS
    log(f"seeding: {n} px x {K} neighbours: triangulate {t_tri:.3f} ms, scale {t_knn:.3f} ms, "
        f"anisotropic frame {t_frame:.3f} ms, "
        f"{res['kept']} kept; {res['roofline']['achieved']:.1f} TFLOP/s FP64 ({res['roofline']['frac']:.2f})")
    return res


def oracle_sample(w, views, cfg, threads):
    """The FP64 CPU oracle on a bounded sample of the workload: forward +
    backward of the given views with the full Gaussian set, on `threads`
    OpenMP threads."""
    import numpy as np
    import oracle
    from paper_2601_00705_amd import scenes
    oracle.set_threads(threads)
    cams = [w["cams"][v] for v in views]
    poses = w["poses"][views]
    ocfg = oracle.Config(tile_w=cfg.tile_w, tile_h=cfg.tile_h, sh_degree=cfg.sh_degree, z_near=cfg.z_near,
                         dilation=cfg.dilation, alpha_min=cfg.alpha_min, alpha_max=cfg.alpha_max,
                         T_min=cfg.T_min, bg=cfg.bg)
    P = sum(c["width"] * c["height"] for c in cams)
    dL = scenes.upstream_grad(5, 3 * P).astype(np.float64)
    t0 = time.perf_counter()
    oracle.render(w["params"], cams, poses, ocfg, want_margin=False)
    oracle.backward(w["params"], cams, poses, ocfg, dL)
    dt = time.perf_counter() - t0
    return P, dt


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, cfg, args):
    """The oracle timed on the host: one thread over the smallest views
    (about 0.4-0.5 Mpix), and every thread the OpenMP runtime has (the box's
    share of cores) over a sample sized to take about as long."""
    import oracle
    cams = w["cams"]
    V = len(cams)
    order = sorted(range(V), key=lambda v: cams[v]["width"] * cams[v]["height"])
    if args.cpu_views:
        views1 = [int(x) for x in args.cpu_views.split(",")]
    else:
        views1, px = [], 0
        for v in order:
            if px >= 400_000:
                break
            views1.append(v)
            px += cams[v]["width"] * cams[v]["height"]
    P1, dt1 = oracle_sample(w, views1, cfg, 1)
    log(f"cpu oracle, 1 thread: {P1 / dt1 / 1e6:.4f} Mpix/s over {dt1:.1f}s")
    nthr = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    # all threads: as many views as one thread's rate predicts for ~10 s of work
    rate1 = P1 / dt1
    budget = rate1 * 10.0 * nthr * 0.7
    viewsN, px = [], 0
    for v in order:
        viewsN.append(v)
        px += cams[v]["width"] * cams[v]["height"]
        if px >= budget:
            break
    PN, dtN = oracle_sample(w, viewsN, cfg, nthr)
    used = oracle.get_threads()
    model = cpu_model()
    log(f"cpu oracle, {used} threads: {PN / dtN / 1e6:.4f} Mpix/s over {dtN:.1f}s ({model})")
    return {"value": PN / dtN / 1e6, "unit": "Mpix/s", "cores": used, "kind": "oracle",
            "sample": f"views {viewsN} ({PN} px) of {w['name']}, fwd+bwd, full Gaussian set, {dtN:.1f} s FP64 "
                      f"on {used} OpenMP threads",
            "cpu_model": model,
            "single_thread": {"value": P1 / dt1 / 1e6, "unit": "Mpix/s", "cores": 1,
                              "sample": f"views {views1} ({P1} px), {dt1:.1f} s"}}


def step_roofline(stage_ms, ms_step, n, sh3, slots_live, pairs, evals, pixels):
    """Step-level roofline: for each stage the time its binding ceiling allows
    (the larger of its algorithmic HBM bytes at 8 TB/s and its FP32
    operations at 157.3 TFLOP/s), summed over the stages and divided by the
    measured step time; also the HBM-only fraction."""
    hbm = HBM_PEAK_GBS * 1e9
    flops = FP32_PEAK_TFLOPS * 1e12
    work = {
        "project": (BYTES_PROJ_PER_GAUSSIAN[sh3] * n + BYTES_PROJ_PER_SLOT * slots_live,
                    OPS_PROJ_PER_SLOT[sh3] * slots_live),
        "bin": (BYTES_BIN_PER_SLOT * slots_live + BYTES_BIN_PER_PAIR * pairs, 0),
        "raster_fwd": (BYTES_RASTER_PER_PAIR * pairs + BYTES_RASTER_PER_PIXEL * pixels, OPS_FWD_PER_EVAL * evals),
        "loss": (BYTES_LOSS_PER_PIXEL * pixels, 0),
        "raster_bwd": (BYTES_RASTER_PER_PAIR * pairs + BYTES_RASTER_PER_PIXEL * pixels, OPS_BWD_PER_EVAL * evals),
        "project_bwd": (BYTES_PBWD_PER_GAUSSIAN[sh3] * n + BYTES_PBWD_PER_SLOT_READ * slots_live,
                        OPS_PBWD_PER_SLOT * slots_live),
    }
    stages, ceil_total, hbm_total = {}, 0.0, 0.0
    for k, (b, o) in work.items():
        t_hbm, t_ops = b / hbm * 1e3, o / flops * 1e3
        ceil = max(t_hbm, t_ops)
        stages[k] = {"ms": stage_ms.get(k), "ceiling_ms": ceil, "bound": "hbm" if t_hbm >= t_ops else "alu",
                     "hbm_bytes": b, "fp32_ops": o}
        ceil_total += ceil
        hbm_total += t_hbm
    return {"frac": ceil_total / ms_step, "ceiling_ms": ceil_total, "hbm_frac": hbm_total / ms_step,
            "stages": stages}


def measure_workload(index, args, torch, steps, warmup, lat_reps, plain_steps, loss="l1", extras=True,
                     precision="fp32", map_order="spatial"):
    """One workload end to end: the batched step captured in a graph and
    replayed (timed), per-view latency, per-kernel time, the blend count, the
    per-view plain launches, and the rooflines.  Returns (result dict,
    workload, cfg, step, renderer)."""
    import numpy as np
    from paper_2601_00705_amd import scenes
    from paper_2601_00705_amd.render import Config, Renderer

    dev = torch.device("cuda:0")
    t_gen = time.time()
    w = scenes.workload(index)
    log(f"workload {w['name']}: generated in {time.time() - t_gen:.1f}s")
    cams = w["cams"]
    n = int(w["params"]["opacity_logit"].shape[0])
    V = len(cams)
    pose_only = [int(x) for x in w["pose_only"]]
    params = {k: torch.from_numpy(v).to(dev) for k, v in w["params"].items()}
    order_desc = "given"
    if map_order == "spatial":
        # the order the map maintenance keeps (untimed here; timed with the
        # maintenance)
        from paper_2601_00705_amd import maintain
        brick = args.brick or maintain.SPATIAL_BRICK
        params = maintain.permute(params, maintain.spatial_order(params["mean"], brick))
        torch.cuda.synchronize()
        order_desc = f"spatial (Morton cells, brick {brick})"
    log(f"map order: {order_desc}")
    poses = torch.from_numpy(w["poses"].astype(np.float32)).to(dev)
    target = target_images(w, params, poses, Config(sh_degree=w["sh_degree"]), Renderer, torch)
    tuned = None
    if args.tile and extras:
        t, _, b = args.tile.lower().partition("/")
        tile = (int(t.split("x")[0]), int(t.split("x")[1]), int(b) if b else 128)
    else:
        from paper_2601_00705_amd import autotune
        tile = None if (args.autotune and extras) else autotune.lookup(cams, n, w["sh_degree"])
        if tile is None:
            tuned = autotune.tune(params, cams, poses, target, w["sh_degree"], pose_only, log=log)
            tile = tuned["best"]
    cfg = Config(tile_w=tile[0], tile_h=tile[1], batch=tile[2], sh_degree=w["sh_degree"],
                 deterministic=args.deterministic, precision=precision)
    log(f"tile {tile[0]}x{tile[1]}, LDS batch {tile[2]}, precision {precision}")
    total_px = sum(c["width"] * c["height"] for c in cams)

    # ---------------- batched: one plan, one graph --------------------
    R, need = sized_renderer(Renderer, n, cams, cfg, params, poses, torch)
    st = Step(R, params, poses, target, pose_only, torch, loss=loss)
    for _ in range(2):
        st.run()
    torch.cuda.synchronize()
    _, ovf = R.pair_count()
    assert not ovf
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        st.run()  # warm the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=cap):
            st.run()
    torch.cuda.synchronize()
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    _, ovf = R.pair_count()
    assert not ovf, "pair capacity exceeded during replay"
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    marks[0].record()
    for k in range(steps):
        graph.replay()
        marks[k + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / steps
    per_step = sorted(marks[k].elapsed_time(marks[k + 1]) for k in range(steps))
    pct = {q: float(np.percentile(per_step, q)) for q in (10, 50, 90)}
    log(f"batched (graph): {ms_step:.3f} ms/step (p10 {pct[10]:.3f}, p50 {pct[50]:.3f}, p90 {pct[90]:.3f}), "
        f"pairs {need}")

    # ---------------- per-view latency: device wall-clock stamps -----------
    # (each replay, the projection stamps the step's start and the last
    # backward tile of each view stamps that view's end; the pose-only views
    # when there are any, else every view)
    lat = []
    po_views = [v for v in range(V) if pose_only[v]]
    sel = po_views or list(range(V))
    for _ in range(lat_reps):
        graph.replay()
        lat.extend(R.view_latency_ms()[sel].tolist())
    view_latency = None
    if lat:
        view_latency = {"views": "pose-only" if po_views else "all", "count": len(sel), "replays": lat_reps,
                        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                        "max_ms": float(np.max(lat))}
        log(f"view latency ({view_latency['views']}, {len(sel)} views x {lat_reps} replays): "
            f"p50 {view_latency['p50_ms']:.3f} ms, p99 {view_latency['p99_ms']:.3f} ms")

    # ---------------- per-kernel device time: library HIP events ----------
    # (eager launches of the same step on the same inputs, right after the
    # timed replays; every group is bracketed on the stream it runs on)
    K = max(3, steps // 2)
    R.set_timing(True)
    for _ in range(K):
        st.run()
    timing = R.read_timing()
    R.set_timing(False)
    kernel_ms = {g: ms / cnt for g, (ms, cnt) in timing.items() if cnt}
    loss_group = {"track": "loss_track", "mapping": "loss_mapping"}.get(loss, "loss_l1")
    stage_ms = {
        "project": kernel_ms["project"],
        "bin": kernel_ms["bin_emit"] + kernel_ms["bin_sort"] + kernel_ms["bin_ranges"],
        "raster_fwd": kernel_ms["raster_fwd"],
        "loss": kernel_ms[loss_group],
        "raster_bwd": kernel_ms["clear_grad2d"] + kernel_ms["raster_bwd"],
        "project_bwd": kernel_ms["project_bwd"],
    }
    log("kernel ms: " + ", ".join(f"{k}={v:.3f}" for k, v in kernel_ms.items()))

    # ---------------- blends / evaluations (untimed counting pass) -----
    nb = torch.empty(total_px, dtype=torch.int32, device=dev)
    R.render_fwd(st.rgb, st.T, st.nc, nb)
    torch.cuda.synchronize()
    blends = int(nb.sum(dtype=torch.int64))
    evals = int(st.nc.sum(dtype=torch.int64))
    slots_live = int((R.records()["geom"][:, 2] >= 0).sum())
    del nb
    log(f"blends {blends}, evaluations (list entries up to the last contributor) {evals}, "
        f"live slots {slots_live}")

    # ---------------- plain: one plan per view, no graph ---------------
    plain = None
    if plain_steps > 0 and V > 1:
        steps_plain = []
        off = 0
        for v in range(V):
            hw = cams[v]["width"] * cams[v]["height"]
            Rv, _ = sized_renderer(Renderer, n, [cams[v]], cfg, params, poses[v:v + 1], torch)
            steps_plain.append(Step(Rv, params, poses[v:v + 1].contiguous(), target[3 * off:3 * (off + hw)],
                                    [pose_only[v]], torch, loss=loss))
            off += hw
        for _ in range(2):
            for s_ in steps_plain:
                s_.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(plain_steps):
            for s_ in steps_plain:
                s_.run()
        torch.cuda.synchronize()
        plain = (time.perf_counter() - t0) * 1e3 / plain_steps
        del steps_plain
        log(f"plain ({V} per-view launch sequences): {plain:.3f} ms/step; speedup {plain / ms_step:.2f}x")

    # ---------------- roofline of the dominant kernel ------------------
    dom = max(kernel_ms, key=kernel_ms.get)
    dom_ms = kernel_ms[dom]
    sh3 = w["sh_degree"] >= 3
    if dom in ("raster_bwd", "raster_fwd"):
        ops = OPS_BWD_PER_EVAL if dom == "raster_bwd" else OPS_FWD_PER_EVAL
        roof = {"bound": "alu", "achieved": evals * ops / (dom_ms * 1e-3) / 1e12, "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "work": f"{ops} FP32 operations x {evals} evaluations"}
    elif dom == "bin_sort":
        algo = need * 24
        roof = {"bound": "hbm", "achieved": algo / (dom_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "work": f"24 B x {need} pairs"}
    else:
        algo = BYTES_PBWD_PER_GAUSSIAN[sh3] * n + BYTES_PBWD_PER_SLOT_READ * slots_live
        roof = {"bound": "hbm", "achieved": algo / (dom_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "work": f"{algo} B"}
    roof["kernel"] = dom
    roof["kernel_ms"] = dom_ms
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom, w["name"], cfg)
    step_roof = step_roofline(stage_ms, ms_step, n, sh3, slots_live, need, evals, total_px)
    log(f"roofline: {dom} {roof['achieved']:.1f} {roof['unit']} ({roof['frac']:.3f} of {roof['peak']}); "
        f"step {step_roof['frac']:.3f} of its ceiling ({step_roof['ceiling_ms']:.3f} ms), "
        f"HBM-only {step_roof['hbm_frac']:.3f}")

    res = {
        "workload": w["name"], "gaussians": n, "views": V, "pixels": total_px, "map_order": order_desc,
        "tile": f"{cfg.tile_w}x{cfg.tile_h}", "batch": cfg.batch, "sh_degree": cfg.sh_degree,
        "ms_per_step": ms_step, "mpix_per_s": total_px / (ms_step * 1e-3) / 1e6,
        "ms_per_step_p10_p50_p90": [pct[10], pct[50], pct[90]],
        "autotune_ms": None if tuned is None else tuned["ms"],
        "blends_per_s": blends / (ms_step * 1e-3), "blends_per_step": blends,
        "evaluations_per_step": evals, "pairs_per_step": need, "live_slots": slots_live,
        "plain_ms_per_step": plain,
        "plain_mpix_per_s": None if plain is None else total_px / (plain * 1e-3) / 1e6,
        "batched_speedup": None if plain is None else plain / ms_step,
        "stage_ms": stage_ms, "kernel_ms": kernel_ms, "roofline": roof, "step_roofline": step_roof,
        "view_latency": view_latency,
    }
    return res, w, cfg, st, R, params, cap


def loss_measurements(torch, st, total_px, reps):
    """The tracking loss (three kernels, HBM bound) and the mapping loss (one
    fused kernel, VALU bound) on the step's render, each replayed from a
    graph of 20 calls (tens of microseconds each: eager launches would time
    the host's launch gaps)."""
    t_ms = _graph_ms(torch, st.track, reps)
    t_bytes = BYTES_TRACK_PER_PIXEL * total_px
    track = {"ms": t_ms, "bound": "hbm", "achieved": t_bytes / (t_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "work": f"{BYTES_TRACK_PER_PIXEL} B x {total_px} px",
             "tau_alpha": TRACK_TAU_ALPHA, "tau_grad": TRACK_TAU_GRAD}
    track["frac"] = track["achieved"] / track["peak"]
    log(f"tracking loss: {t_ms:.4f} ms, {track['achieved']:.0f} GB/s ({track['frac']:.2f} of HBM)")

    m_ms = _graph_ms(torch, st.mapping, reps)
    m_slots = SLOTS_MAP_PER_PIXEL * total_px
    mapl = {"ms": m_ms, "bound": "alu", "achieved": m_slots / (m_ms * 1e-3) / 1e12, "peak": VALU_PEAK_TSLOTS,
            "unit": "T VALU slots/s", "work": f"{SLOTS_MAP_PER_PIXEL} slots x {total_px} px",
            "hbm_GBs": BYTES_MAP_PER_PIXEL * total_px / (m_ms * 1e-3) / 1e9, "lambda": MAP_LAMBDA}
    mapl["frac"] = mapl["achieved"] / mapl["peak"]
    log(f"mapping loss: {m_ms:.4f} ms, {mapl['achieved']:.1f} T slots/s ({mapl['frac']:.2f} of VALU issue), "
        f"{mapl['hbm_GBs']:.0f} GB/s")

    return track, mapl


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the renderer is benchmarked on a single MI355X "
              "(multi-GPU view sharding is a design note, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")

    if args.copy_probe:
        # plain device copy of a known size (scales the HBM byte counters)
        a = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("copy probe: 3 x 256 MiB device copies")

    res, w, cfg, st, R, params, cap = measure_workload(
        args.config, args, torch, args.steps, args.warmup, max(100, args.steps),
        0 if args.no_plain else args.steps, loss=args.loss, precision=args.precision, map_order=args.map_order)
    total_px = res["pixels"]

    # ---------------- tracking loss: its three kernels, HBM bound -----------
    # (tens of microseconds each, so they are replayed from a graph of 20
    # calls: eager launches would time the host's launch gaps)
    reps = max(3, args.steps // 4)
    track = mapl = None
    if args.precision == "fp32" and not args.no_extras:
        track, mapl = loss_measurements(torch, st, total_px, reps)

    # ---------------- seeding and map maintenance at the workload's size ----
    seed_res = None if args.no_seeding else seeding_measurement(torch, max(3, args.steps // 4), log)
    maint = None if args.no_extras else maintenance_measurement(torch, w, params, st.T, R.cams,
                                                                max(3, args.steps // 4), log)

    # ---------------- CPU baseline: the oracle on a bounded sample -----
    cpu = None if args.no_cpu_baseline else cpu_baseline(w, cfg, args)
    del st, R, params
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    # ---------------- the mixed-precision variant on the same workload ------
    # (32-byte staging records with binary16 colour, binary16 image; the same
    # graph-replayed step with the L1 seed)
    mixed = None
    if not args.no_mixed and args.loss == "l1":
        mres, *_ = measure_workload(args.config, args, torch, args.steps, args.warmup, 0, 0, loss="l1",
                                   extras=False, precision="mixed")
        mixed = {"ms_per_step": mres["ms_per_step"], "mpix_per_s": mres["mpix_per_s"],
                 "speedup_vs_fp32": res["ms_per_step"] / mres["ms_per_step"], "kernel_ms": mres["kernel_ms"]}
        log(f"mixed precision: {mres['ms_per_step']:.3f} ms/step ({mixed['speedup_vs_fp32']:.3f}x the fp32 step)")
        del mres
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

    # ---------------- the same step on the generator's order ---------------
    given = None
    if args.map_order == "spatial" and not args.no_given:
        gres, *_ = measure_workload(args.config, args, torch, args.steps, args.warmup, 0, 0, loss=args.loss,
                                   extras=False, precision=args.precision, map_order="given")
        given = {"ms_per_step": gres["ms_per_step"], "mpix_per_s": gres["mpix_per_s"],
                 "spatial_speedup": gres["ms_per_step"] / res["ms_per_step"], "kernel_ms": gres["kernel_ms"]}
        log(f"generator's order: {gres['ms_per_step']:.3f} ms/step (the spatial order is "
            f"{given['spatial_speedup']:.3f}x faster)")
        del gres
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

    # ---------------- the 3M-Gaussian tracking-and-mapping batch ----------
    # (a compact second leg: 4 mapping views at 1920x1080 and 32 pose-only
    # solves at 640x480 in one graph, per-solve latency over 100 replays)
    second = None
    if args.config != 4 and not args.no_second:
        second, *_ = measure_workload(4, args, torch, min(args.steps, 10), 3, 100, 3, loss="l1", extras=False,
                                      map_order=args.map_order)
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

    out = {
        "metric": "fwd+bwd Mpix/s and Gaussian-pixel blends/s, batched vs plain, 1 MI355X",
        "value": res["mpix_per_s"],
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f32+f16",
        "data": "synthetic",
        "config": {"workload": res["workload"], "gaussians": res["gaussians"], "views": res["views"],
                   "pixels": total_px, "tile": res["tile"], "batch": res["batch"], "sh_degree": res["sh_degree"],
                   "mode": "batched-graph", "loss": args.loss, "deterministic": bool(args.deterministic),
                   "map_order": res["map_order"]},
        "autotune_ms": res["autotune_ms"],
        "ms_per_step_p10_p50_p90": res["ms_per_step_p10_p50_p90"],
        "blends_per_s": res["blends_per_s"],
        "blends_per_step": res["blends_per_step"],
        "evaluations_per_step": res["evaluations_per_step"],
        "pairs_per_step": res["pairs_per_step"],
        "plain_ms_per_step": res["plain_ms_per_step"],
        "plain_mpix_per_s": res["plain_mpix_per_s"],
        "batched_speedup": res["batched_speedup"],
        "stage_ms": res["stage_ms"],
        "kernel_ms": res["kernel_ms"],
        "roofline": res["roofline"],
        "step_roofline": res["step_roofline"],
        "view_latency": res["view_latency"],
        "tracking_loss": track,
        "mapping_loss": mapl,
        "seeding": seed_res,
        "maintenance": maint,
        "cpu_baseline": cpu,
        "mixed_precision": mixed,
        "given_order": given,
        "track_map_3M": second,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
