"""Torch-facing renderer: plans, workspaces and a torch.autograd.Function.

PyTorch provides device memory and streams; every computation is a call into
libgsr (see include/gsr.h).  ``Renderer`` owns one plan (host object) and its
workspace (a uint8 CUDA tensor); ``render`` is differentiable w.r.t. every
Gaussian parameter and the pose twists xi (the left update T <- exp(xi^) T of
Eq. (leftupdate), gradient at xi = 0).
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import lib

PARAM_KEYS = ("mean", "quat", "log_scale", "opacity_logit", "colour")


@dataclass
class Config:
    """Renderer settings.  Defaults: 16x16 tiles, near plane 0.2, screen
    covariance dilation 0.3 px^2, alpha in [1/255, 0.99], early stop at
    T < 1e-4, black background, RGB colour, FP64-atomic backward (set
    deterministic for the bitwise-reproducible fixed-point one), float32
    staging records and images (precision "mixed": 32-byte records with
    binary16 colour and binary16 images)."""
    tile_w: int = 16
    tile_h: int = 16
    batch: int = 128
    sh_degree: int = -1
    z_near: float = 0.2
    dilation: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    bg: tuple = (0.0, 0.0, 0.0)
    deterministic: bool = False
    precision: str = "fp32"


def _stream(device):
    return torch.cuda.current_stream(device).cuda_stream


class Renderer:
    """One plan + workspace for n Gaussians and a fixed set of cameras."""

    def __init__(self, n, cams, cfg: Config = Config(), pair_capacity=None, device="cuda"):
        self.n = int(n)
        self.cams = [dict(c) for c in cams]
        self.cfg = cfg
        self.device = torch.device(device)
        self.total_pixels = sum(int(c["width"]) * int(c["height"]) for c in cams)
        if pair_capacity is None:
            # a first guess; forward_all grows it to the measured need
            pair_capacity = min(max(1 << 16, 8 * self.n * len(cams)), 1 << 26)
        self.plan = None
        # bumped whenever the workspace's records, pair lists or capacity
        # change (projection, plan growth); the autograd Function compares it
        # to decide whether its forward's state is still in the workspace
        self.generation = 0
        self._make(int(min(pair_capacity, (1 << 32) - 1)))

    def _make(self, capacity):
        self.generation += 1
        if self.plan is not None:
            lib.gsr_plan_destroy(self.plan)
        self.plan = lib.gsr_plan_create(self.n, self.cams, self.cfg, capacity)
        self.capacity = capacity
        nbytes = lib.gsr_plan_workspace_bytes(self.plan)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        lib.gsr_plan_bind(self.plan, self.workspace, _stream(self.device))
        self.layout = lib.gsr_plan_layout(self.plan)
        self.info = lib.gsr_plan_get_info(self.plan)

    def __del__(self):
        plan, self.plan = getattr(self, "plan", None), None
        if plan is not None and lib is not None and getattr(lib, "_lib", None) is not None:
            try:
                lib.gsr_plan_destroy(plan)
            except Exception:  # interpreter shutdown
                pass

    # -- views into the workspace (for tests and diagnostics) -------------
    def _view(self, off, count, dtype):
        nbytes = count * torch.empty((), dtype=dtype).element_size()
        return self.workspace[off:off + nbytes].view(dtype)

    def records(self):
        S = self.info.slots
        L = self.layout
        return {
            "geom": self._view(L.geom, 4 * S, torch.float32).view(S, 4),
            "conic_o": self._view(L.conic_o, 4 * S, torch.float32).view(S, 4),
            "rgb_d": self._view(L.rgb_d, 4 * S, torch.float32).view(S, 4),
            "qthr": self._view(L.qthr, S, torch.float32),
            "grad2d": self._view(L.grad2d, 9 * S, torch.float64).view(S, 9),
            # bit k of word [w][v] set when slot (v, 64 w + k) is live
            "live_mask": self._view(L.live_mask, len(self.cams) * ((self.n + 63) // 64),
                                    torch.int64).view(-1, len(self.cams)),
        }

    def stamps(self):
        """Device wall-clock ticks [V + 1]: when the last backward tile of
        each view finished, then when the last projection began (int64 view
        into the workspace; read after a synchronisation)."""
        V = len(self.cams)
        return self._view(self.layout.stamps, V + 1, torch.int64)

    def view_latency_ms(self):
        """Per-view latency of the last step in ms: completion of the view's
        backward minus the start of the projection (synchronises)."""
        torch.cuda.synchronize(self.device)
        s = self.stamps().cpu().double()
        return ((s[:-1] - s[-1]) / lib.gsr_device_clock_hz() * 1e3)

    def sorted_pairs(self, count):
        L = self.layout
        return (self._view(L.keys, count, torch.int64), self._view(L.vals, count, torch.int32),
                self._view(L.ranges, 2 * self.info.total_tiles, torch.int32).view(-1, 2))

    # -- the C ABI calls ---------------------------------------------------
    def gaussians(self, params):
        return lib.make_gaussians(self.n, *(params[k] for k in PARAM_KEYS))

    def project(self, params, poses):
        self.generation += 1
        lib.gsr_project(self.plan, self.gaussians(params), poses, _stream(self.device))

    def bin(self):
        lib.gsr_bin(self.plan, _stream(self.device))

    def pair_count(self):
        return lib.gsr_pair_count(self.plan, _stream(self.device))

    @property
    def image_dtype(self):
        """dtype of the rendered image: float32, or float16 for a mixed plan."""
        return torch.float16 if self.cfg.precision == "mixed" else torch.float32

    def new_image_buffers(self, want_blend=False):
        P = self.total_pixels
        dev = self.device
        return (torch.empty(3 * P, dtype=self.image_dtype, device=dev), torch.empty(P, device=dev),
                torch.empty(P, dtype=torch.int32, device=dev),
                torch.empty(P, dtype=torch.int32, device=dev) if want_blend else None)

    def render_fwd(self, rgb, T_final, n_contrib, n_blend=None):
        lib.gsr_render_fwd(self.plan, rgb, T_final, n_contrib, n_blend, _stream(self.device))

    def loss_l1(self, rgb, target, dL_drgb):
        lib.gsr_loss_l1(self.plan, rgb, target, dL_drgb, _stream(self.device))

    def loss_track(self, rgb, T_final, target, tau_alpha, tau_grad, loss, exposure, dL_drgb, dL_dT=None):
        """Tracking loss per view (loss [V] and exposure [V][2] float64) and
        its gradient seed dL_drgb / dL_dT for render_bwd."""
        lib.gsr_loss_track(self.plan, rgb, T_final, target, tau_alpha, tau_grad, loss, exposure, dL_drgb, dL_dT,
                           _stream(self.device))

    def loss_mapping(self, rgb, target, lam, loss, dL_drgb):
        """Mapping loss (1 - lam) L1 + lam (1 - SSIM) over all views (loss [1]
        float64) and its gradient seed dL_drgb for render_bwd."""
        lib.gsr_loss_mapping(self.plan, rgb, target, lam, loss, dL_drgb, _stream(self.device))

    def render_bwd(self, params, poses, T_final, n_contrib, dL_drgb, dL_dT=None, pose_only=None, grads=None,
                   d_xi=None):
        g = None if grads is None else lib.Grads(*(lib._p(grads[k]) for k in PARAM_KEYS))
        lib.gsr_render_bwd(self.plan, self.gaussians(params), poses, T_final, n_contrib, dL_drgb, dL_dT,
                           pose_only, g, d_xi, _stream(self.device))

    def raster_bwd(self, T_final, n_contrib, dL_drgb, dL_dT=None):
        lib.gsr_raster_bwd(self.plan, T_final, n_contrib, dL_drgb, dL_dT, _stream(self.device))

    def project_bwd(self, params, poses, pose_only=None, grads=None, d_xi=None):
        g = None if grads is None else lib.Grads(*(lib._p(grads[k]) for k in PARAM_KEYS))
        lib.gsr_project_bwd(self.plan, self.gaussians(params), poses, pose_only, g, d_xi, _stream(self.device))

    def set_timing(self, enable):
        """Per-launch-group HIP-event timing inside the library (eager launches only)."""
        lib.gsr_plan_set_timing(self.plan, enable)

    def read_timing(self):
        """{group: (total ms, launches)} since timing was switched on."""
        return lib.gsr_plan_read_timing(self.plan)

    def forward_all(self, params, poses, want_blend=False, grow=True):
        """project + bin (+ capacity growth) + render_fwd; returns buffers."""
        self.project(params, poses)
        self.bin()
        if grow:
            need, ovf = self.pair_count()
            if ovf:
                self._make(int(min(need * 5 // 4 + 4096, (1 << 32) - 1)))
                self.project(params, poses)
                self.bin()
        out = self.new_image_buffers(want_blend)
        self.render_fwd(*out)
        return out


def split_views(flat, cams, channels):
    """Concatenated per-view buffer -> list of [C, H, W] (or [H, W]) views."""
    out, off = [], 0
    for c in cams:
        hw = int(c["width"]) * int(c["height"])
        chunk = flat[off * channels:(off + hw) * channels]
        out.append(chunk.view(channels, int(c["height"]), int(c["width"])) if channels > 1
                   else chunk.view(int(c["height"]), int(c["width"])))
        off += hw
    return out


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, renderer, poses, pose_only, xi, mean, quat, log_scale, opacity_logit, colour):
        params = dict(zip(PARAM_KEYS, (mean, quat, log_scale, opacity_logit, colour)))
        params = {k: v.contiguous() for k, v in params.items()}
        poses = poses.contiguous()
        rgb, T, nc, _ = renderer.forward_all(params, poses)
        ctx.renderer = renderer
        ctx.generation = renderer.generation
        ctx.pose_only = pose_only
        ctx.save_for_backward(poses, T, nc, *(params[k] for k in PARAM_KEYS))
        ctx.mark_non_differentiable(nc)
        return rgb, T, nc

    @staticmethod
    def backward(ctx, d_rgb, d_T, _d_nc):
        r = ctx.renderer
        poses, T, nc, *tensors = ctx.saved_tensors
        params = dict(zip(PARAM_KEYS, tensors))
        if r.generation != ctx.generation:
            # another forward (or a plan growth) has run on this renderer since
            # this one: its sorted lists and staging records are gone from the
            # workspace.  Projection and binning are deterministic, so running
            # them again on the saved inputs restores exactly this forward's
            # state (the capacity only grows, so it still fits).
            r.project(params, poses)
            r.bin()
        grads = {k: torch.empty_like(v) for k, v in params.items()}
        d_xi = torch.empty(len(r.cams), 6, device=poses.device)
        d_rgb = (torch.zeros(3 * r.total_pixels, device=poses.device) if d_rgb is None
                 else d_rgb.to(torch.float32).contiguous())  # float32 also for a binary16 image
        d_T = None if d_T is None else d_T.contiguous()
        r.render_bwd(params, poses, T, nc, d_rgb, d_T, ctx.pose_only, grads, d_xi)
        return (None, None, None, d_xi, grads["mean"], grads["quat"], grads["log_scale"],
                grads["opacity_logit"], grads["colour"])


def render(renderer: Renderer, params, poses, xi=None, pose_only=None):
    """Differentiable render of all views of ``renderer``.

    params: dict of CUDA float32 planes; poses: [V, 12] world-to-camera;
    xi: optional [V, 6] twist placeholder (zeros, requires_grad) whose
    gradient is dL/dxi at xi = 0.  Returns (rgb [sum 3HW], T_final [sum HW],
    n_contrib [sum HW]); use split_views for per-view images."""
    if xi is None:
        xi = torch.zeros(len(renderer.cams), 6, device=poses.device)
    return _RenderFn.apply(renderer, poses, pose_only, xi, *(params[k] for k in PARAM_KEYS))
