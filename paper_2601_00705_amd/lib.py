"""ctypes binding of libgsr.so (the C ABI in include/gsr.h).

Argument marshalling only: every step of the renderer runs in the library's
HIP kernels.  Importing this module loads the library and raises if it has
not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsr.so")
MAX_VIEWS = 64

OK, EINVAL, ECAPACITY, EHIP, EUNSUPPORTED, ESTATE = 0, -1, -2, -3, -4, -5


class GsrError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        super().__init__(f"{where}: {_lib.gsr_status_str(status).decode()} (status {status})"
                         + (f": {detail}" if detail else ""))


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


class Config(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("sh_degree", ctypes.c_int32), ("z_near", ctypes.c_float), ("dilation", ctypes.c_float),
                ("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float), ("T_min", ctypes.c_float),
                ("bg", ctypes.c_float * 3), ("deterministic", ctypes.c_int32), ("precision", ctypes.c_int32)]


class Gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("mean", ctypes.c_void_p), ("quat", ctypes.c_void_p),
                ("log_scale", ctypes.c_void_p), ("opacity_logit", ctypes.c_void_p),
                ("colour", ctypes.c_void_p)]


class Grads(ctypes.Structure):
    _fields_ = [("d_mean", ctypes.c_void_p), ("d_quat", ctypes.c_void_p), ("d_log_scale", ctypes.c_void_p),
                ("d_opacity_logit", ctypes.c_void_p), ("d_colour", ctypes.c_void_p)]


class Layout(ctypes.Structure):
    _fields_ = [(k, ctypes.c_size_t) for k in
                ("counters", "geom", "conic_o", "rgb_d", "qthr", "stage", "grad2d", "keys", "vals", "ranges",
                 "stamps", "live_mask", "total")]


class SeedView(ctypes.Structure):
    _fields_ = [("P", ctypes.c_double * 12), ("centre", ctypes.c_double * 3), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("image", ctypes.c_void_p), ("gain", ctypes.c_double),
                ("bias", ctypes.c_double)]


class SeedConfig(ctypes.Structure):
    _fields_ = [("max_reproj", ctypes.c_double), ("min_parallax", ctypes.c_double),
                ("alpha_lo", ctypes.c_double), ("alpha_hi", ctypes.c_double)]


class Planes(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("mean", "quat", "log_scale", "opacity_logit", "colour")]


class AdamConfig(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float * 5), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_float), ("max_grad_norm", ctypes.c_float), ("ema", ctypes.c_float),
                ("step", ctypes.c_int32)]


class PruneConfig(ctypes.Structure):
    _fields_ = [("m_min", ctypes.c_int32), ("v_min", ctypes.c_float), ("sigma_max", ctypes.c_float),
                ("alpha_min", ctypes.c_float)]


ADAM_WORKSPACE_BYTES = 16384


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("slots", ctypes.c_int64), ("capacity", ctypes.c_int64),
                ("total_pixels", ctypes.c_int64), ("n_views", ctypes.c_int32),
                ("total_tiles", ctypes.c_int32), ("sort_passes", ctypes.c_int32),
                ("tile_bits", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2601_00705_amd.build.build() "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    st = ctypes.c_int
    sigs = {
        "gsr_plan_create": (st, [ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_int64, P]),
        "gsr_plan_destroy": (None, [P]),
        "gsr_plan_workspace_bytes": (ctypes.c_size_t, [P]),
        "gsr_plan_bind": (st, [P, P, ctypes.c_size_t, P]),
        "gsr_plan_layout": (st, [P, P]),
        "gsr_plan_get_info": (st, [P, P]),
        "gsr_project": (st, [P, P, P, P]),
        "gsr_bin": (st, [P, P]),
        "gsr_render_fwd": (st, [P, P, P, P, P, P]),
        "gsr_loss_l1": (st, [P, P, P, P, P]),
        "gsr_loss_track": (st, [P, P, P, P, ctypes.c_double, ctypes.c_double, P, P, P, P, P]),
        "gsr_loss_mapping": (st, [P, P, P, ctypes.c_double, P, P, P]),
        "gsr_render_bwd": (st, [P, P, P, P, P, P, P, P, P, P, P]),
        "gsr_raster_bwd": (st, [P, P, P, P, P, P]),
        "gsr_project_bwd": (st, [P, P, P, P, P, P, P]),
        "gsr_pair_count": (st, [P, P, P, P]),
        "gsr_seed_triangulate": (st, [ctypes.c_int64, ctypes.c_int32, P, P, P, P, P, P, P, P, P, P, P, P, P, P]),
        "gsr_seed_scale_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64]),
        "gsr_seed_scale": (st, [ctypes.c_int64, P, P, ctypes.c_float, P, ctypes.c_size_t, P, P]),
        "gsr_adam_step": (st, [ctypes.c_int64, ctypes.c_int32, P, P, P, P, P, P, P, P, P]),
        "gsr_covis": (st, [ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_float, P, P, P]),
        "gsr_prune_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64]),
        "gsr_prune": (st, [ctypes.c_int64, P, P, P, P, P, P, P, P, P]),
        "gsr_prune_noalloc": (st, [ctypes.c_int64, P, P, P, P, P, P, P, P]),
        "gsr_compact": (st, [ctypes.c_int64, ctypes.c_int32, P, P, P, P, P]),
        "gsr_seed_frame": (st, [ctypes.c_int64, P, P, P, P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_float,
                                P, ctypes.c_size_t, P, P, P]),
        "gsr_nearest": (st, [ctypes.c_int64, P, P, P, ctypes.c_size_t, P, P]),
        "gsr_merge": (st, [ctypes.c_int64, ctypes.c_int32, P, P, P, ctypes.c_double, ctypes.c_double, P, P, P]),
        "gsr_keep_list": (st, [ctypes.c_int64, P, P, P, P, P]),
        "gsr_spatial_order_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64]),
        "gsr_spatial_order": (st, [ctypes.c_int64, P, ctypes.c_int32, P, P, ctypes.c_size_t, P]),
        "gsr_device_clock_hz": (st, [P]),
        "gsr_plan_set_timing": (st, [P, ctypes.c_int32]),
        "gsr_plan_read_timing": (st, [P, ctypes.c_int32, P, P]),
        "gsr_status_str": (ctypes.c_char_p, [st]),
        "gsr_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
EXPORTS = ("gsr_plan_create", "gsr_plan_destroy", "gsr_plan_workspace_bytes", "gsr_plan_bind",
           "gsr_plan_layout", "gsr_plan_get_info", "gsr_project", "gsr_bin", "gsr_render_fwd",
           "gsr_loss_l1", "gsr_loss_track", "gsr_loss_mapping", "gsr_render_bwd", "gsr_raster_bwd", "gsr_project_bwd", "gsr_pair_count",
           "gsr_plan_set_timing", "gsr_plan_read_timing", "gsr_status_str", "gsr_last_error",
           "gsr_seed_triangulate", "gsr_seed_scale_workspace_bytes", "gsr_seed_scale",
           "gsr_adam_step", "gsr_covis", "gsr_prune_workspace_bytes", "gsr_prune", "gsr_prune_noalloc", "gsr_compact",
           "gsr_nearest", "gsr_merge", "gsr_keep_list", "gsr_seed_frame", "gsr_device_clock_hz",
           "gsr_spatial_order_workspace_bytes", "gsr_spatial_order")

# gsr_config.precision: float32 staging records and images, or the mixed
# variant (32-byte records with binary16 colour, binary16 images)
PRECISIONS = {"fp32": 0, "mixed": 1}

# launch groups of gsr_plan_read_timing (gsr_timer)
TIMERS = ("project", "bin_emit", "bin_sort", "bin_ranges", "raster_fwd", "loss_l1", "clear_grad2d",
          "raster_bwd", "project_bwd", "loss_track", "loss_mapping")


def raw():
    """The loaded ctypes library."""
    return _lib


def check(status, where):
    if status != OK:
        raise GsrError(status, where, _lib.gsr_last_error().decode())
    return status


def _p(x):
    """Device pointer of a tensor (or None)."""
    return None if x is None else ctypes.c_void_p(x.data_ptr())


def make_cameras(cams):
    arr = (Camera * len(cams))()
    for k, c in enumerate(cams):
        arr[k] = Camera(int(c["width"]), int(c["height"]), float(c["fx"]), float(c["fy"]),
                        float(c["cx"]), float(c["cy"]))
    return arr


def make_config(cfg):
    c = Config()
    c.tile_w, c.tile_h, c.batch, c.sh_degree = cfg.tile_w, cfg.tile_h, getattr(cfg, "batch", 0), cfg.sh_degree
    c.z_near, c.dilation = cfg.z_near, cfg.dilation
    c.alpha_min, c.alpha_max, c.T_min = cfg.alpha_min, cfg.alpha_max, cfg.T_min
    for k in range(3):
        c.bg[k] = float(cfg.bg[k])
    c.deterministic = 1 if getattr(cfg, "deterministic", False) else 0
    prec = getattr(cfg, "precision", "fp32")
    if prec not in PRECISIONS:
        raise ValueError(f"precision must be one of {tuple(PRECISIONS)}")
    c.precision = PRECISIONS[prec]
    return c


def make_gaussians(n, mean, quat, log_scale, opacity_logit, colour):
    return Gaussians(int(n), _p(mean), _p(quat), _p(log_scale), _p(opacity_logit), _p(colour))


def gsr_plan_create(n, cams, cfg, pair_capacity):
    plan = ctypes.c_void_p()
    cam_arr = make_cameras(cams)
    ccfg = make_config(cfg)
    check(_lib.gsr_plan_create(int(n), len(cams), ctypes.cast(cam_arr, ctypes.c_void_p),
                               ctypes.byref(ccfg), int(pair_capacity), ctypes.byref(plan)),
          "gsr_plan_create")
    return plan


def gsr_plan_destroy(plan):
    _lib.gsr_plan_destroy(plan)


def gsr_plan_workspace_bytes(plan):
    return int(_lib.gsr_plan_workspace_bytes(plan))


def gsr_plan_bind(plan, workspace, stream):
    check(_lib.gsr_plan_bind(plan, _p(workspace), workspace.numel() * workspace.element_size(),
                             ctypes.c_void_p(stream)), "gsr_plan_bind")


def gsr_plan_layout(plan):
    lay = Layout()
    check(_lib.gsr_plan_layout(plan, ctypes.byref(lay)), "gsr_plan_layout")
    return lay


def gsr_plan_get_info(plan):
    info = PlanInfo()
    check(_lib.gsr_plan_get_info(plan, ctypes.byref(info)), "gsr_plan_get_info")
    return info


def gsr_project(plan, g: Gaussians, poses, stream):
    return check(_lib.gsr_project(plan, ctypes.byref(g), _p(poses), ctypes.c_void_p(stream)), "gsr_project")


def gsr_bin(plan, stream):
    return check(_lib.gsr_bin(plan, ctypes.c_void_p(stream)), "gsr_bin")


def gsr_render_fwd(plan, rgb, T_final, n_contrib, n_blend, stream):
    return check(_lib.gsr_render_fwd(plan, _p(rgb), _p(T_final), _p(n_contrib), _p(n_blend),
                                     ctypes.c_void_p(stream)), "gsr_render_fwd")


def gsr_loss_l1(plan, rgb, target, dL_drgb, stream):
    return check(_lib.gsr_loss_l1(plan, _p(rgb), _p(target), _p(dL_drgb), ctypes.c_void_p(stream)),
                 "gsr_loss_l1")


def gsr_loss_track(plan, rgb, T_final, target, tau_alpha, tau_grad, loss, exposure, dL_drgb, dL_dT, stream):
    return check(_lib.gsr_loss_track(plan, _p(rgb), _p(T_final), _p(target), ctypes.c_double(tau_alpha),
                                     ctypes.c_double(tau_grad), _p(loss), _p(exposure), _p(dL_drgb), _p(dL_dT),
                                     ctypes.c_void_p(stream)), "gsr_loss_track")


def gsr_loss_mapping(plan, rgb, target, lam, loss, dL_drgb, stream):
    return check(_lib.gsr_loss_mapping(plan, _p(rgb), _p(target), ctypes.c_double(lam), _p(loss), _p(dL_drgb),
                                       ctypes.c_void_p(stream)), "gsr_loss_mapping")


def gsr_seed_triangulate(views, cfg, x_ref, x_nb, kappa, mean, colour, opacity_logit, valid, best, err, angle,
                         kappa_bar, stream):
    """views: list of dicts (P [3][4], centre [3], width, height, image (device tensor), gain, bias);
    cfg: dict (max_reproj, min_parallax, alpha_lo, alpha_hi)."""
    arr = (SeedView * len(views))()
    for k, v in enumerate(views):
        arr[k].P = (ctypes.c_double * 12)(*[float(x) for x in list(v["P"].reshape(-1))])
        arr[k].centre = (ctypes.c_double * 3)(*[float(x) for x in v["centre"]])
        arr[k].width, arr[k].height = int(v["width"]), int(v["height"])
        arr[k].image = ctypes.c_void_p(v["image"].data_ptr())
        arr[k].gain, arr[k].bias = float(v["gain"]), float(v["bias"])
    c = SeedConfig(float(cfg["max_reproj"]), float(cfg["min_parallax"]), float(cfg["alpha_lo"]),
                   float(cfg["alpha_hi"]))
    n = int(x_ref.shape[-1])
    return check(_lib.gsr_seed_triangulate(n, len(views) - 1, arr, ctypes.byref(c), _p(x_ref), _p(x_nb), _p(kappa),
                                           _p(mean), _p(colour), _p(opacity_logit), _p(valid), _p(best), _p(err),
                                           _p(angle), _p(kappa_bar), ctypes.c_void_p(stream)),
                 "gsr_seed_triangulate")


def gsr_seed_scale_workspace_bytes(n):
    return int(_lib.gsr_seed_scale_workspace_bytes(int(n)))


def gsr_seed_scale(n, mean, valid, floor_scale, workspace, log_scale, stream):
    return check(_lib.gsr_seed_scale(int(n), _p(mean), _p(valid), ctypes.c_float(floor_scale), _p(workspace),
                                     workspace.numel() * workspace.element_size(), _p(log_scale),
                                     ctypes.c_void_p(stream)), "gsr_seed_scale")


PLANES = ("mean", "quat", "log_scale", "opacity_logit", "colour")


def _planes(d):
    return Planes(*(d[k].data_ptr() for k in PLANES))


def gsr_device_clock_hz():
    hz = ctypes.c_double()
    check(_lib.gsr_device_clock_hz(ctypes.byref(hz)), "gsr_device_clock_hz")
    return hz.value


def gsr_adam_step(n, colour_rows, params, grads, m, v, anchor, cfg: AdamConfig, workspace, norm, stream):
    """params, grads, m, v: dicts of device tensors over PLANES."""
    pp, gg, mm, vv = _planes(params), _planes(grads), _planes(m), _planes(v)
    return check(_lib.gsr_adam_step(int(n), int(colour_rows), ctypes.byref(pp), ctypes.byref(gg), ctypes.byref(mm),
                                    ctypes.byref(vv), _p(anchor), ctypes.byref(cfg), _p(workspace), _p(norm),
                                    ctypes.c_void_p(stream)), "gsr_adam_step")


def gsr_covis(pixels, n_frames, T_key, T_frames, tau, counts, iou, stream):
    return check(_lib.gsr_covis(int(pixels), int(n_frames), _p(T_key), _p(T_frames), ctypes.c_float(tau),
                                _p(counts), _p(iou), ctypes.c_void_p(stream)), "gsr_covis")


def gsr_prune_workspace_bytes(n):
    return int(_lib.gsr_prune_workspace_bytes(int(n)))


def gsr_prune(n, m_obs, v_vis, log_scale, opacity_logit, cfg: PruneConfig, keep_index, kept, workspace, stream):
    return check(_lib.gsr_prune(int(n), _p(m_obs), _p(v_vis), _p(log_scale), _p(opacity_logit), ctypes.byref(cfg),
                                _p(keep_index), _p(kept), _p(workspace), ctypes.c_void_p(stream)), "gsr_prune")


def gsr_prune_noalloc(n, m_obs, v_vis, log_scale, opacity_logit, cfg: PruneConfig, keep_index, kept, stream):
    """gsr_prune without a workspace (the library's fixed device scratch;
    n <= PRUNE_NOALLOC_MAX_N)."""
    return check(_lib.gsr_prune_noalloc(int(n), _p(m_obs), _p(v_vis), _p(log_scale), _p(opacity_logit),
                                        ctypes.byref(cfg), _p(keep_index), _p(kept), ctypes.c_void_p(stream)),
                 "gsr_prune_noalloc")


PRUNE_NOALLOC_MAX_N = 1 << 27


def gsr_compact(n, rows, src, keep_index, kept, dst, stream):
    return check(_lib.gsr_compact(int(n), int(rows), _p(src), _p(keep_index), _p(kept), _p(dst),
                                  ctypes.c_void_p(stream)), "gsr_compact")


def gsr_render_bwd(plan, g: Gaussians, poses, T_final, n_contrib, dL_drgb, dL_dT, pose_only, grads, d_xi,
                   stream):
    po = None
    if pose_only is not None:
        po = (ctypes.c_uint8 * len(pose_only))(*[int(x) for x in pose_only])
    gp = ctypes.byref(grads) if grads is not None else None
    return check(_lib.gsr_render_bwd(plan, ctypes.byref(g), _p(poses), _p(T_final), _p(n_contrib),
                                     _p(dL_drgb), _p(dL_dT),
                                     ctypes.cast(po, ctypes.c_void_p) if po is not None else None,
                                     gp, _p(d_xi), ctypes.c_void_p(stream)), "gsr_render_bwd")


def _pose_only_arg(pose_only):
    if pose_only is None:
        return None
    po = (ctypes.c_uint8 * len(pose_only))(*[int(x) for x in pose_only])
    return po


def gsr_raster_bwd(plan, T_final, n_contrib, dL_drgb, dL_dT, stream):
    return check(_lib.gsr_raster_bwd(plan, _p(T_final), _p(n_contrib), _p(dL_drgb), _p(dL_dT),
                                     ctypes.c_void_p(stream)), "gsr_raster_bwd")


def gsr_project_bwd(plan, g: Gaussians, poses, pose_only, grads, d_xi, stream):
    po = _pose_only_arg(pose_only)
    return check(_lib.gsr_project_bwd(plan, ctypes.byref(g), _p(poses),
                                      ctypes.cast(po, ctypes.c_void_p) if po is not None else None,
                                      ctypes.byref(grads) if grads is not None else None, _p(d_xi),
                                      ctypes.c_void_p(stream)), "gsr_project_bwd")


def gsr_pair_count(plan, stream):
    req = ctypes.c_int64()
    ovf = ctypes.c_int32()
    s = _lib.gsr_pair_count(plan, ctypes.byref(req), ctypes.byref(ovf), ctypes.c_void_p(stream))
    if s not in (OK, ECAPACITY):
        check(s, "gsr_pair_count")
    return int(req.value), bool(ovf.value)


def gsr_plan_set_timing(plan, enable):
    check(_lib.gsr_plan_set_timing(plan, 1 if enable else 0), "gsr_plan_set_timing")


def gsr_plan_read_timing(plan):
    """{group: (total ms, launches)} for every launch group (waits for the
    recorded events)."""
    out = {}
    for k, name in enumerate(TIMERS):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        check(_lib.gsr_plan_read_timing(plan, k, ctypes.byref(ms), ctypes.byref(cnt)), "gsr_plan_read_timing")
        out[name] = (ms.value, cnt.value)
    return out


def gsr_nearest(n, mean, valid, workspace, nn_index, stream):
    return check(_lib.gsr_nearest(int(n), _p(mean), _p(valid), _p(workspace),
                                  workspace.numel() * workspace.element_size(), _p(nn_index),
                                  ctypes.c_void_p(stream)), "gsr_nearest")


def gsr_merge(n, colour_rows, params, v_vis, nn_index, radius, colour_tol, out, keep, stream):
    pin, pout = _planes(params), _planes(out)
    return check(_lib.gsr_merge(int(n), int(colour_rows), ctypes.byref(pin), _p(v_vis), _p(nn_index),
                                ctypes.c_double(radius), ctypes.c_double(colour_tol), ctypes.byref(pout), _p(keep),
                                ctypes.c_void_p(stream)), "gsr_merge")


def gsr_keep_list(n, mask, keep_index, kept, workspace, stream):
    return check(_lib.gsr_keep_list(int(n), _p(mask), _p(keep_index), _p(kept), _p(workspace),
                                    ctypes.c_void_p(stream)), "gsr_keep_list")


def gsr_spatial_order_workspace_bytes(n):
    return int(_lib.gsr_spatial_order_workspace_bytes(int(n)))


def gsr_spatial_order(n, mean, brick, index, workspace, stream):
    return check(_lib.gsr_spatial_order(int(n), _p(mean), int(brick), _p(index), _p(workspace),
                                        workspace.numel() * workspace.element_size(), ctypes.c_void_p(stream)),
                 "gsr_spatial_order")


def gsr_seed_frame(n, mean, valid, err, angle, P_ref, centre_ref, radius, c_par, floor_scale, workspace, quat,
                   log_scale, stream):
    P = (ctypes.c_double * 12)(*[float(x) for x in P_ref])
    c = (ctypes.c_double * 3)(*[float(x) for x in centre_ref])
    return check(_lib.gsr_seed_frame(int(n), _p(mean), _p(valid), _p(err), _p(angle), P, c, ctypes.c_double(radius),
                                     ctypes.c_double(c_par), ctypes.c_float(floor_scale), _p(workspace),
                                     workspace.numel() * workspace.element_size(), _p(quat), _p(log_scale),
                                     ctypes.c_void_p(stream)), "gsr_seed_frame")
