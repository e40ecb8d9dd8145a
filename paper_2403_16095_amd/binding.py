"""ctypes binding of the C ABI declared in include/cgsr.h.

Argument marshalling only: every function here forwards to the symbol of the
same name in ``libcgsr.so``.  Device pointers are passed as Python ints (a
torch tensor's ``data_ptr()``), streams as ints (``torch.cuda.Stream.cuda_stream``).
The library must be built (``paper_2403_16095_amd.build.build()``); there is no
fallback of any kind when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcgsr.so")

CGSR_OK = 0
CGSR_ERR_INVALID_ARG = -1
CGSR_ERR_OOM = -2
CGSR_ERR_HIP = -3
CGSR_ERR_CAPACITY = -4
CGSR_ERR_STATE = -5
CGSR_MAX_VIEWS = 64

STATUS_NAMES = {0: "CGSR_OK", -1: "CGSR_ERR_INVALID_ARG", -2: "CGSR_ERR_OOM", -3: "CGSR_ERR_HIP",
                -4: "CGSR_ERR_CAPACITY", -5: "CGSR_ERR_STATE"}

EXPORTED = (
    "cgsr_default_settings", "cgsr_state_create", "cgsr_state_destroy", "cgsr_state_reserve",
    "cgsr_render", "cgsr_render_nu", "cgsr_nu_prune", "cgsr_mapping_objective", "cgsr_gaussian_adam_step",
    "cgsr_backward", "cgsr_tracking_loss_grad", "cgsr_mapping_loss_grad", "cgsr_pose_adam_step",
    "cgsr_tracking_step", "cgsr_autotune_tracking", "cgsr_autotune_render", "cgsr_spawn_gaussians",
    "cgsr_compact_gaussians", "cgsr_compact_gaussians_noalloc", "cgsr_set_densify_stats", "cgsr_densify_gaussians",
    "cgsr_state_check", "cgsr_get_stats", "cgsr_get_timings", "cgsr_time_tracking_blend", "cgsr_debug_buffers",
    "cgsr_debug_tile_order", "cgsr_last_error", "cgsr_version",
)
STAGES = ("project", "emit", "sort", "blend_fwd", "blend_bwd", "project_bwd")


class CgsrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class cgsr_camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float)]


class cgsr_gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", C.c_void_p), ("log_scales", C.c_void_p),
                ("quats", C.c_void_p), ("opacity_logits", C.c_void_p), ("rgb", C.c_void_p),
                ("sh", C.c_void_p), ("sh_degree", C.c_int32)]


class cgsr_gaussian_arrays(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("rgb", C.c_void_p), ("sh", C.c_void_p), ("sh_degree", C.c_int32)]


class cgsr_images(C.Structure):
    _fields_ = [("color", C.c_void_p), ("depth", C.c_void_p), ("opacity", C.c_void_p),
                ("depth_median", C.c_void_p), ("uncertainty", C.c_void_p)]


cgsr_image_grads = cgsr_images  # same layout, const on the C side


class cgsr_gaussian_grads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("rgb", C.c_void_p), ("sh", C.c_void_p)]


class cgsr_settings(C.Structure):
    _fields_ = [("sync_capacity", C.c_int32), ("timing", C.c_int32), ("fwd_pixels_per_lane", C.c_int32),
                ("bwd_pixels_per_lane", C.c_int32), ("count_work", C.c_int32)]


class cgsr_adam_params(C.Structure):
    _fields_ = [("lr_rho", C.c_float), ("lr_phi", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float)]


class cgsr_mapping_weights(C.Structure):
    _fields_ = [("color", C.c_float), ("ssim", C.c_float), ("geo", C.c_float), ("align", C.c_float),
                ("iso", C.c_float), ("var", C.c_float), ("iso_epsilon", C.c_float)]


class cgsr_gaussian_adam_params(C.Structure):
    _fields_ = [("lr_means", C.c_float), ("lr_log_scales", C.c_float), ("lr_quats", C.c_float),
                ("lr_opacity_logits", C.c_float), ("lr_rgb", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("lr_sh_rest", C.c_float), ("sh_degree", C.c_int32)]


class cgsr_stats(C.Structure):
    _fields_ = [("visible", C.c_int64), ("pairs", C.c_int64), ("pair_capacity", C.c_int64),
                ("overflow", C.c_int32), ("n_views", C.c_int32), ("processed", C.c_int64),
                ("blended", C.c_int64), ("walked", C.c_int64), ("peak_pairs", C.c_int64)]


_lib = None


def lib() -> C.CDLL:
    """Load libcgsr.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime under the same soname as ROCm's; loading
    # it first makes libcgsr.so bind to that one instance, so device pointers
    # and streams from torch are valid here.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2403_16095_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    st = C.c_int
    vp = C.c_void_p
    L.cgsr_default_settings.argtypes = [C.POINTER(cgsr_settings)]
    L.cgsr_default_settings.restype = None
    L.cgsr_state_create.argtypes = [C.POINTER(cgsr_settings), C.POINTER(vp)]
    L.cgsr_state_destroy.argtypes = [vp]
    L.cgsr_state_reserve.argtypes = [vp, C.c_int64, C.c_int64, C.c_int64, C.c_int64]
    L.cgsr_render.argtypes = [vp, C.POINTER(cgsr_gaussians), C.c_int32, vp, C.POINTER(cgsr_camera),
                              C.POINTER(vp), C.POINTER(cgsr_images), vp]
    L.cgsr_render_nu.argtypes = [vp, C.POINTER(cgsr_gaussians), C.c_int32, vp, C.POINTER(cgsr_camera),
                                 C.POINTER(vp), C.POINTER(cgsr_images), C.POINTER(vp), vp, vp, vp]
    L.cgsr_mapping_objective.argtypes = [vp, C.POINTER(cgsr_mapping_weights), C.POINTER(cgsr_images), C.POINTER(vp),
                                         C.POINTER(vp), C.POINTER(cgsr_images), vp, vp, vp]
    L.cgsr_gaussian_adam_step.argtypes = [C.c_int64, C.POINTER(cgsr_gaussian_grads), C.POINTER(cgsr_gaussian_grads),
                                          vp, vp, C.POINTER(cgsr_gaussian_adam_params), vp]
    L.cgsr_nu_prune.argtypes = [C.c_int64, vp, vp, C.c_float, C.c_float, vp, vp, vp, vp]
    L.cgsr_backward.argtypes = [vp, C.POINTER(cgsr_images), C.POINTER(cgsr_gaussian_grads), vp, vp]
    L.cgsr_tracking_loss_grad.argtypes = [C.c_int32, C.c_int32, vp, vp, vp, vp, C.c_float, C.c_float, vp, vp,
                                          vp, vp]
    L.cgsr_mapping_loss_grad.argtypes = [C.c_int32, C.c_int32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.cgsr_pose_adam_step.argtypes = [C.c_int32, vp, vp, vp, C.POINTER(cgsr_adam_params), vp]
    L.cgsr_tracking_step.argtypes = [vp, C.POINTER(cgsr_gaussians), C.c_int32, vp, C.POINTER(cgsr_camera),
                                     C.POINTER(vp), C.POINTER(vp), C.c_float, C.c_float, vp, vp,
                                     C.POINTER(cgsr_adam_params), vp, vp]
    L.cgsr_autotune_tracking.argtypes = [vp, C.POINTER(cgsr_gaussians), C.c_int32, vp, C.POINTER(cgsr_camera),
                                         C.POINTER(vp), C.POINTER(vp), C.c_int32, C.POINTER(cgsr_settings), vp]
    L.cgsr_autotune_render.argtypes = [vp, C.POINTER(cgsr_gaussians), C.c_int32, vp, C.POINTER(cgsr_camera),
                                       C.POINTER(vp), C.POINTER(cgsr_images), C.POINTER(cgsr_images),
                                       C.POINTER(cgsr_gaussian_grads), vp, C.c_int32, C.POINTER(cgsr_settings), vp]
    L.cgsr_spawn_gaussians.argtypes = [C.POINTER(cgsr_gaussian_arrays), C.c_int64, C.c_int64, C.POINTER(cgsr_camera),
                                       vp, vp, vp, vp, C.c_float, C.c_int32, C.c_float, C.POINTER(C.c_int64), vp]
    L.cgsr_compact_gaussians.argtypes = [C.c_int64, vp, C.POINTER(cgsr_gaussian_arrays),
                                         C.POINTER(cgsr_gaussian_arrays), C.c_int32, C.POINTER(vp), C.POINTER(vp),
                                         C.POINTER(C.c_int32), C.POINTER(C.c_int64), vp]
    L.cgsr_compact_gaussians_noalloc.argtypes = L.cgsr_compact_gaussians.argtypes
    L.cgsr_set_densify_stats.argtypes = [vp, vp, vp]
    L.cgsr_densify_gaussians.argtypes = [C.c_int64, vp, vp, C.c_float, C.c_float, vp,
                                         C.POINTER(cgsr_gaussian_arrays), C.POINTER(cgsr_gaussian_arrays), C.c_int64,
                                         C.POINTER(C.c_int64), vp]
    L.cgsr_state_check.argtypes = [vp, vp]
    L.cgsr_get_stats.argtypes = [vp, vp, C.POINTER(cgsr_stats)]
    L.cgsr_get_timings.argtypes = [vp, C.POINTER(C.c_float)]
    L.cgsr_time_tracking_blend.argtypes = [vp, C.c_int32, vp, C.POINTER(C.c_float)]
    L.cgsr_debug_buffers.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                     C.POINTER(vp)]
    L.cgsr_debug_tile_order.argtypes = [vp, C.POINTER(vp), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.cgsr_last_error.argtypes = []
    L.cgsr_last_error.restype = C.c_char_p
    L.cgsr_version.argtypes = []
    L.cgsr_version.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("cgsr_default_settings", "cgsr_last_error", "cgsr_version"):
            getattr(L, name).restype = st
    _lib = L
    return L


def _check(status: int) -> None:
    if status != CGSR_OK:
        raise CgsrError(status, lib().cgsr_last_error().decode())


def cgsr_default_settings() -> cgsr_settings:
    s = cgsr_settings()
    lib().cgsr_default_settings(C.byref(s))
    return s


def cgsr_state_create(settings: cgsr_settings | None = None) -> int:
    out = C.c_void_p()
    _check(lib().cgsr_state_create(C.byref(settings) if settings is not None else None, C.byref(out)))
    return out.value


def cgsr_state_destroy(state: int) -> None:
    _check(lib().cgsr_state_destroy(state))


def cgsr_state_reserve(state: int, max_records: int, max_pixels: int, max_tiles: int, max_tile_pairs: int) -> None:
    _check(lib().cgsr_state_reserve(state, max_records, max_pixels, max_tiles, max_tile_pairs))


def cgsr_render(state: int, g: cgsr_gaussians, n_views: int, poses: int, cams, depth_obs, outs,
                stream: int) -> None:
    """cams: sequence of cgsr_camera; depth_obs: sequence of device pointers (0/None) or None;
    outs: sequence of cgsr_images."""
    cam_arr = (cgsr_camera * n_views)(*cams)
    out_arr = (cgsr_images * n_views)(*outs)
    dep = None if depth_obs is None else (C.c_void_p * n_views)(*[p or None for p in depth_obs])
    _check(lib().cgsr_render(state, C.byref(g), n_views, poses, cam_arr, dep, out_arr, stream))


def cgsr_render_nu(state: int, g: cgsr_gaussians, n_views: int, poses: int, cams, depth_obs, outs, dominant,
                   nu_sum, nu_count, stream: int) -> None:
    """depth_obs: sequence of device pointers (required); dominant: sequence of
    device pointers (0/None allowed) or None."""
    cam_arr = (cgsr_camera * n_views)(*cams)
    out_arr = (cgsr_images * n_views)(*outs)
    dep = (C.c_void_p * n_views)(*depth_obs)
    dom = None if dominant is None else (C.c_void_p * n_views)(*[p or None for p in dominant])
    _check(lib().cgsr_render_nu(state, C.byref(g), n_views, poses, cam_arr, dep, out_arr, dom, nu_sum, nu_count,
                                stream))


def cgsr_mapping_objective(state: int, weights: cgsr_mapping_weights, maps, target_color, target_depth, dimgs,
                           dlog_scales, loss, stream: int) -> None:
    """maps, dimgs: sequences of cgsr_images; target_color/target_depth:
    sequences of device pointers (0/None allowed) or None."""
    n = len(maps)
    m_arr = (cgsr_images * n)(*maps)
    d_arr = (cgsr_images * n)(*dimgs)
    tc = None if target_color is None else (C.c_void_p * n)(*[p or None for p in target_color])
    td = None if target_depth is None else (C.c_void_p * n)(*[p or None for p in target_depth])
    _check(lib().cgsr_mapping_objective(state, C.byref(weights), m_arr, tc, td, d_arr, dlog_scales, loss, stream))


def cgsr_gaussian_adam_step(n, params: cgsr_gaussian_grads, grads: cgsr_gaussian_grads, moments, step,
                            hp: cgsr_gaussian_adam_params, stream) -> None:
    _check(lib().cgsr_gaussian_adam_step(n, C.byref(params), C.byref(grads), moments, step, C.byref(hp), stream))


def cgsr_spawn_gaussians(dst: cgsr_gaussian_arrays, n, capacity, cam: cgsr_camera, pose, color, depth, opacity, psi,
                         stride, init_logit, stream) -> int:
    """Returns n plus the number spawned."""
    out = C.c_int64(0)
    _check(lib().cgsr_spawn_gaussians(C.byref(dst), n, capacity, C.byref(cam), pose, color, depth, opacity, psi,
                                      stride, init_logit, C.byref(out), stream))
    return out.value


def cgsr_compact_gaussians(n, keep, src: cgsr_gaussian_arrays, dst: cgsr_gaussian_arrays, extra_src, extra_dst,
                           extra_width, stream) -> int:
    """extra_*: sequences of device pointers and widths (may be empty)."""
    k = len(extra_src)
    es = (C.c_void_p * max(k, 1))(*extra_src)
    ed = (C.c_void_p * max(k, 1))(*extra_dst)
    ew = (C.c_int32 * max(k, 1))(*extra_width)
    out = C.c_int64(0)
    _check(lib().cgsr_compact_gaussians(n, keep, C.byref(src), C.byref(dst), k, es, ed, ew, C.byref(out), stream))
    return out.value


def cgsr_compact_gaussians_noalloc(n, keep, src: cgsr_gaussian_arrays, dst: cgsr_gaussian_arrays, extra_src,
                                   extra_dst, extra_width, stream) -> int:
    """As cgsr_compact_gaussians, with the library's fixed scratch (no device allocation)."""
    k = len(extra_src)
    es = (C.c_void_p * max(k, 1))(*extra_src)
    ed = (C.c_void_p * max(k, 1))(*extra_dst)
    ew = (C.c_int32 * max(k, 1))(*extra_width)
    out = C.c_int64(0)
    _check(lib().cgsr_compact_gaussians_noalloc(n, keep, C.byref(src), C.byref(dst), k, es, ed, ew, C.byref(out),
                                                stream))
    return out.value


def cgsr_set_densify_stats(state: int, grad_accum, count) -> None:
    _check(lib().cgsr_set_densify_stats(state, grad_accum, count))


def cgsr_densify_gaussians(n, grad_accum, count, grad_threshold, dense_scale, normals, src: cgsr_gaussian_arrays,
                           dst: cgsr_gaussian_arrays, capacity, stream) -> int:
    out = C.c_int64(0)
    _check(lib().cgsr_densify_gaussians(n, grad_accum, count, grad_threshold, dense_scale, normals, C.byref(src),
                                        C.byref(dst), capacity, C.byref(out), stream))
    return out.value


def cgsr_nu_prune(n, nu_sum, nu_count, tau, low_opacity, opacity_logits, nu, n_pruned, stream) -> None:
    _check(lib().cgsr_nu_prune(n, nu_sum, nu_count, tau, low_opacity, opacity_logits, nu, n_pruned, stream))


def cgsr_backward(state: int, dimgs, dG: cgsr_gaussian_grads | None, dposes: int | None, stream: int) -> None:
    arr = (cgsr_images * len(dimgs))(*dimgs)
    _check(lib().cgsr_backward(state, arr, C.byref(dG) if dG is not None else None, dposes, stream))


def cgsr_tracking_loss_grad(width, height, color, depth, target_color, target_depth, lambda_color, lambda_depth,
                            dcolor, ddepth, loss, stream) -> None:
    _check(lib().cgsr_tracking_loss_grad(width, height, color, depth, target_color, target_depth, lambda_color,
                                         lambda_depth, dcolor, ddepth, loss, stream))


def cgsr_mapping_loss_grad(width, height, color, depth, uncertainty, target_color, target_depth, dcolor, ddepth,
                           duncertainty, loss, stream) -> None:
    _check(lib().cgsr_mapping_loss_grad(width, height, color, depth, uncertainty, target_color, target_depth, dcolor,
                                        ddepth, duncertainty, loss, stream))


def cgsr_pose_adam_step(n_views, poses, dposes, adam, params: cgsr_adam_params, stream) -> None:
    _check(lib().cgsr_pose_adam_step(n_views, poses, dposes, adam, C.byref(params), stream))


def cgsr_tracking_step(state: int, g: cgsr_gaussians, n_views: int, poses: int, cams, target_color, target_depth,
                       lambda_color: float, lambda_depth: float, dposes, adam, params, loss, stream: int) -> None:
    """cams: sequence of cgsr_camera; target_color/target_depth: sequences of device pointers."""
    cam_arr = (cgsr_camera * n_views)(*cams)
    tc = (C.c_void_p * n_views)(*target_color)
    td = (C.c_void_p * n_views)(*target_depth)
    _check(lib().cgsr_tracking_step(state, C.byref(g), n_views, poses, cam_arr, tc, td, lambda_color, lambda_depth,
                                    dposes, adam, C.byref(params) if params is not None else None, loss, stream))


def cgsr_autotune_tracking(state: int, g: cgsr_gaussians, n_views: int, poses: int, cams, target_color,
                           target_depth, repeats: int, stream: int) -> cgsr_settings:
    cam_arr = (cgsr_camera * n_views)(*cams)
    tc = (C.c_void_p * n_views)(*target_color)
    td = (C.c_void_p * n_views)(*target_depth)
    out = cgsr_settings()
    _check(lib().cgsr_autotune_tracking(state, C.byref(g), n_views, poses, cam_arr, tc, td, repeats, C.byref(out),
                                        stream))
    return out


def cgsr_autotune_render(state: int, g: cgsr_gaussians, n_views: int, poses: int, cams, depth_obs, outs, dimgs,
                         dG: cgsr_gaussian_grads | None, dposes: int | None, repeats: int,
                         stream: int) -> cgsr_settings:
    """depth_obs: sequence of device pointers (0/None allowed) or None; outs, dimgs: sequences of cgsr_images."""
    cam_arr = (cgsr_camera * n_views)(*cams)
    out_arr = (cgsr_images * n_views)(*outs)
    grad_arr = (cgsr_images * n_views)(*dimgs)
    dep = None if depth_obs is None else (C.c_void_p * n_views)(*[p or None for p in depth_obs])
    out = cgsr_settings()
    _check(lib().cgsr_autotune_render(state, C.byref(g), n_views, poses, cam_arr, dep, out_arr, grad_arr,
                                      C.byref(dG) if dG is not None else None, dposes, repeats, C.byref(out), stream))
    return out


def cgsr_state_check(state: int, stream: int) -> None:
    _check(lib().cgsr_state_check(state, stream))


def cgsr_get_stats(state: int, stream: int) -> cgsr_stats:
    out = cgsr_stats()
    _check(lib().cgsr_get_stats(state, stream, C.byref(out)))
    return out


def cgsr_get_timings(state: int) -> dict:
    """Stage durations (ms) of the last timed render and backward."""
    out = (C.c_float * len(STAGES))()
    _check(lib().cgsr_get_timings(state, out))
    return dict(zip(STAGES, [float(v) for v in out]))


def cgsr_time_tracking_blend(state: int, reps: int, stream: int) -> float:
    """Average ms of one re-run of the last tracking step's fused blend kernel."""
    out = C.c_float(0.0)
    _check(lib().cgsr_time_tracking_blend(state, reps, stream, C.byref(out)))
    return out.value


def cgsr_debug_buffers(state: int):
    ptrs = [C.c_void_p() for _ in range(5)]
    _check(lib().cgsr_debug_buffers(state, *[C.byref(p) for p in ptrs]))
    return [p.value for p in ptrs]


def cgsr_debug_tile_order(state: int):
    """(device pointer or None, tiles, kept) of the last render's tile order."""
    ptr, tiles, kept = C.c_void_p(), C.c_int32(), C.c_int32()
    _check(lib().cgsr_debug_tile_order(state, C.byref(ptr), C.byref(tiles), C.byref(kept)))
    return ptr.value, tiles.value, kept.value


def cgsr_last_error() -> str:
    return lib().cgsr_last_error().decode()


def cgsr_version() -> str:
    return lib().cgsr_version().decode()
