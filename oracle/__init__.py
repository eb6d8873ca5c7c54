"""FP64 CPU oracle of the differentiable Gaussian-splatting renderer.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers; the product path never imports it.

The arithmetic lives in ``gsr_oracle.c`` (plain C, double precision) and is
written from the paper's equations: Eq. (proj) for the projected mean and EWA
covariance, Eq. (alpha) for front-to-back compositing, the appendix's
covariance parameterisation R diag(s^2) R^T and Eq. (app-sh) for colour, and
Eqs. (leftupdate), (muCjac), (muIjac), (sigmaIjac) for the pose tangent.
``brute.py`` is a second, NumPy-only forward used to pin the tiled C forward
on tiny inputs.  This module only marshals arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "gsr_oracle.c")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction; OpenMP
    over pixel rows, Gaussians and tile lists)."""
    if force or not os.path.exists(_LIB_PATH):
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
            "-ffp-contract=off", "-fno-fast-math", "-Wall", "-o", _LIB_PATH, _SRC, "-lm",
        ])
    return _LIB_PATH


@dataclass
class Config:
    """Renderer settings; defaults are the readings the oracle takes where the
    paper is silent (tile size, dilation eps, alpha bounds, T_min, bg)."""
    tile_w: int = 16
    tile_h: int = 16
    sh_degree: int = -1
    z_near: float = 0.2
    dilation: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    bg: tuple = (0.0, 0.0, 0.0)
    # tolerance model only (the "clear" ratio): the renderer under test
    # stages the projected centre and conic rounded to float32
    staging_f32: bool = False


class _CConfig(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("sh_degree", ctypes.c_int32),
                ("z_near", ctypes.c_double), ("dilation", ctypes.c_double),
                ("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("T_min", ctypes.c_double), ("bg", ctypes.c_double * 3), ("staging_f32", ctypes.c_int32)]


class _CCamera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double)]


class _CScene(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("mean", ctypes.c_void_p), ("quat", ctypes.c_void_p),
                ("log_scale", ctypes.c_void_p), ("opacity_logit", ctypes.c_void_p),
                ("colour", ctypes.c_void_p)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _lib.or_render.restype = ctypes.c_int
        _lib.or_backward.restype = ctypes.c_int
        _lib.or_project.restype = ctypes.c_int
        _lib.or_bin_f32.restype = ctypes.c_int64
        _lib.or_get_threads.restype = ctypes.c_int32
    return _lib


def power2_error_bound(u, v, A, B, C, px, py, xc, yc, p2, staging_f32=False):
    """The oracle's bound on the float32 error of the exp2-space power at a
    pixel, expanded about the tile centre (xc, yc) (test tolerance model);
    staging_f32: the centre and conic are rounded to float32 first."""
    f = _load().or_power2_error
    f.restype = ctypes.c_double
    f.argtypes = [ctypes.c_double] * 10 + [ctypes.c_int32]
    return float(f(u, v, A, B, C, px, py, xc, yc, p2, 1 if staging_f32 else 0))


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops (results differ across thread
    counts only by FP64 rounding: per-thread partial sums are merged in
    thread order)."""
    _load().or_set_threads(ctypes.c_int32(int(n)))


def get_threads() -> int:
    return int(_load().or_get_threads())


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _cfg(cfg: Config) -> _CConfig:
    c = _CConfig()
    c.tile_w, c.tile_h, c.sh_degree = cfg.tile_w, cfg.tile_h, cfg.sh_degree
    c.z_near, c.dilation = cfg.z_near, cfg.dilation
    c.alpha_min, c.alpha_max, c.T_min = cfg.alpha_min, cfg.alpha_max, cfg.T_min
    for k in range(3):
        c.bg[k] = float(cfg.bg[k])
    c.staging_f32 = 1 if cfg.staging_f32 else 0
    return c


def _cams(cams):
    arr = (_CCamera * len(cams))()
    for k, cam in enumerate(cams):
        arr[k].width, arr[k].height = int(cam["width"]), int(cam["height"])
        arr[k].fx, arr[k].fy = float(cam["fx"]), float(cam["fy"])
        arr[k].cx, arr[k].cy = float(cam["cx"]), float(cam["cy"])
    return arr


class _Scene:
    """Keeps float64 contiguous copies alive while C reads them."""

    def __init__(self, params):
        self.mean = np.ascontiguousarray(params["mean"], dtype=np.float64)
        self.quat = np.ascontiguousarray(params["quat"], dtype=np.float64)
        self.log_scale = np.ascontiguousarray(params["log_scale"], dtype=np.float64)
        self.opacity_logit = np.ascontiguousarray(params["opacity_logit"], dtype=np.float64)
        self.colour = np.ascontiguousarray(params["colour"], dtype=np.float64)
        self.n = self.opacity_logit.shape[0]
        self.c = _CScene(self.n, _ptr(self.mean), _ptr(self.quat), _ptr(self.log_scale),
                         _ptr(self.opacity_logit), _ptr(self.colour))


def n_pixels(cams):
    return int(sum(int(c["width"]) * int(c["height"]) for c in cams))


def split_views(flat, cams, channels):
    """Split a concatenated per-view buffer into [C, H, W] (or [H, W]) arrays."""
    out, off = [], 0
    for cam in cams:
        hw = int(cam["width"]) * int(cam["height"])
        chunk = flat[off * channels:(off + hw) * channels]
        shape = (channels, int(cam["height"]), int(cam["width"])) if channels > 1 else (
            int(cam["height"]), int(cam["width"]))
        out.append(chunk.reshape(shape))
        off += hw
    return out


def render(params, cams, poses, cfg: Config = Config(), want_margin=True):
    """Forward render.  Returns flat concatenated buffers: rgb [sum 3*H*W],
    T_final, n_contrib, n_blend, margin and clear [sum H*W].

    margin: the smallest relative distance of any of the pixel's decisions
    (alpha_min skip, alpha_max clamp, T_min stop) from its threshold.
    clear: the smallest ratio of that distance to a bound on the float32
    error of the quantity compared (a tolerance model for the tests, see
    power2_abs_error in gsr_oracle.c); a pixel with clear > 1 takes every
    decision the same way in float32."""
    lib = _load()
    sc = _Scene(params)
    poses = np.ascontiguousarray(poses, dtype=np.float64).reshape(-1, 12)
    P = n_pixels(cams)
    rgb = np.zeros(3 * P)
    T = np.zeros(P)
    nc = np.zeros(P, dtype=np.int32)
    nb = np.zeros(P, dtype=np.int32)
    mg = np.zeros(P) if want_margin else None
    cl = np.zeros(P) if want_margin else None
    ccfg = _cfg(cfg)
    rc = lib.or_render(ctypes.byref(sc.c), ctypes.c_int32(len(cams)), _cams(cams), _ptr(poses),
                       ctypes.byref(ccfg), _ptr(rgb), _ptr(T), _ptr(nc), _ptr(nb), _ptr(mg), _ptr(cl))
    if rc != 0:
        raise RuntimeError("oracle render failed")
    return {"rgb": rgb, "T_final": T, "n_contrib": nc, "n_blend": nb, "margin": mg, "clear": cl}


def backward(params, cams, poses, cfg: Config, dL_drgb, dL_dT=None, pose_only=None,
             want_grad2d=False):
    """Analytic backward of ``render`` for an upstream gradient."""
    lib = _load()
    sc = _Scene(params)
    poses = np.ascontiguousarray(poses, dtype=np.float64).reshape(-1, 12)
    V = len(cams)
    n = sc.n
    dL_drgb = np.ascontiguousarray(dL_drgb, dtype=np.float64)
    dL_dT = None if dL_dT is None else np.ascontiguousarray(dL_dT, dtype=np.float64)
    po = None if pose_only is None else np.ascontiguousarray(pose_only, dtype=np.uint8)
    out = {
        "mean": np.zeros((3, n)), "quat": np.zeros((4, n)), "log_scale": np.zeros((3, n)),
        "opacity_logit": np.zeros(n), "colour": np.zeros(sc.colour.shape),
        "xi": np.zeros((V, 6)),
    }
    g2 = np.zeros((V, n, 9)) if want_grad2d else None
    g2a = np.zeros((V, n, 9)) if want_grad2d else None
    ccfg = _cfg(cfg)
    rc = lib.or_backward(ctypes.byref(sc.c), ctypes.c_int32(V), _cams(cams), _ptr(poses),
                         ctypes.byref(ccfg), _ptr(dL_drgb), _ptr(dL_dT), _ptr(po),
                         _ptr(out["mean"]), _ptr(out["quat"]), _ptr(out["log_scale"]),
                         _ptr(out["opacity_logit"]), _ptr(out["colour"]), _ptr(out["xi"]),
                         _ptr(g2), _ptr(g2a))
    if rc != 0:
        raise RuntimeError("oracle backward failed")
    if want_grad2d:
        # screen-space gradients per (view, Gaussian): d(u, v, A, B, C, o, r,
        # g, b), and the sums of their addends' magnitudes (their ratio to
        # the magnitude of the sum measures cancellation)
        out["grad2d"] = g2
        out["grad2d_abs"] = g2a
    return out


PROJ_FIELDS = ["valid", "u", "v", "A", "B", "C", "o", "r", "g", "b", "depth", "rx", "ry",
               "cov_a", "cov_b", "cov_c", "mcx", "mcy", "mcz", "tx0", "ty0", "tx1", "ty1"]


def project(params, cam, pose, cfg: Config):
    """Per-Gaussian projected record in FP64, as a dict of arrays."""
    lib = _load()
    sc = _Scene(params)
    pose = np.ascontiguousarray(pose, dtype=np.float64).reshape(12)
    out = np.zeros((sc.n, len(PROJ_FIELDS)))
    ccfg = _cfg(cfg)
    lib.or_project(ctypes.byref(sc.c), _cams([cam]), _ptr(pose), ctypes.byref(ccfg), _ptr(out))
    return {k: out[:, j] for j, k in enumerate(PROJ_FIELDS)}


def bin_f32(cams, n, u, v, rx, ry, A, B, C, qthr, depth, tile_w, tile_h):
    """Reference binning of float32 records (slot = view * n + i) into sorted
    (tile | depth-bits) keys, slot values and per-tile ranges."""
    lib = _load()
    arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (u, v, rx, ry, A, B, C, qthr, depth)]
    V = len(cams)
    W = np.array([c["width"] for c in cams], dtype=np.int32)
    H = np.array([c["height"] for c in cams], dtype=np.int32)
    tiles = int(sum(((w + tile_w - 1) // tile_w) * ((h + tile_h - 1) // tile_h) for w, h in zip(W, H)))
    ranges = np.zeros(2 * tiles, dtype=np.uint32)
    M = lib.or_bin_f32(ctypes.c_int32(V), _ptr(W), _ptr(H), ctypes.c_int64(n), *(_ptr(a) for a in arrs),
                       ctypes.c_int32(tile_w), ctypes.c_int32(tile_h), ctypes.c_int64(0), None, None,
                       _ptr(ranges))
    keys = np.zeros(max(M, 1), dtype=np.uint64)
    vals = np.zeros(max(M, 1), dtype=np.uint32)
    lib.or_bin_f32(ctypes.c_int32(V), _ptr(W), _ptr(H), ctypes.c_int64(n), *(_ptr(a) for a in arrs),
                   ctypes.c_int32(tile_w), ctypes.c_int32(tile_h), ctypes.c_int64(M), _ptr(keys), _ptr(vals),
                   _ptr(ranges))
    return keys[:M], vals[:M], ranges.reshape(tiles, 2)


def sh_basis(deg, direction):
    """Real SH basis values Y_k(direction) for k < (deg+1)^2, Eq. (app-sh)."""
    lib = _load()
    d = np.ascontiguousarray(direction, dtype=np.float64)
    Y = np.zeros(16)
    lib.or_sh_basis(ctypes.c_int32(deg), _ptr(d), _ptr(Y))
    return Y[: (deg + 1) ** 2]


from .track import track_loss, track_view, grad_norm as track_grad_norm, exposure as track_exposure  # noqa: E402
from . import seed as seeding  # noqa: E402
from . import ssim  # noqa: E402,F401
from . import optim  # noqa: E402,F401
