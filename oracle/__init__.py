"""FP64 CPU oracle of the CG-SLAM Gaussian rasterizer -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The product path (the HIP library and its Python
binding) never does, and the two share no code.

The heavy lifting is plain C in ``cgsr_oracle.c`` (Eq. 1-10 of the paper and
their chain rule, in double precision).  This module marshals numpy arrays
into it and adds the small host-side pieces of the method written directly
from their definitions: the L1 losses (Eq. 14, 16, 19), their gradient
images, Adam and the pose retraction used by sequential tracking (Eq. 20).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)


class _Gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", _dp), ("log_scales", _dp), ("quats", _dp),
                ("opacity_logits", _dp), ("rgb", _dp), ("sh", _dp), ("sh_degree", C.c_int32)]


class _Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double),
                ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double)]


class _Pose(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3)]


class _Projection(C.Structure):
    _fields_ = [("visible", _ip), ("clamp", _ip), ("p_cam", _dp), ("mu", _dp), ("cov2d", _dp),
                ("conic", _dp), ("depth", _dp), ("opacity", _dp), ("rect", _ip),
                ("rect_edges", _dp)]


class _Images(C.Structure):
    _fields_ = [("color", _dp), ("depth", _dp), ("opacity", _dp), ("depth_median", _dp),
                ("uncertainty", _dp), ("n_contrib", _ip), ("t_final", _dp), ("median_id", _ip),
                ("decision_margin", _dp), ("order_margin", _dp), ("stop_order_margin", _dp)]


class _ImageGrads(C.Structure):
    _fields_ = [("color", _dp), ("depth", _dp), ("opacity", _dp), ("depth_median", _dp),
                ("uncertainty", _dp)]


class _Grads(C.Structure):
    _fields_ = [("means", _dp), ("log_scales", _dp), ("quats", _dp), ("opacity_logits", _dp),
                ("rgb", _dp), ("pose", _dp), ("sh", _dp), ("mu", _dp), ("conic", _dp), ("opacity", _dp),
                ("depth", _dp)]


def lib():
    """Load (building first if needed) the oracle's shared library."""
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        _lib = C.CDLL(path)
        _lib.orc_project.argtypes = [C.POINTER(_Gaussians), C.POINTER(_Camera), C.POINTER(_Pose),
                                     C.POINTER(_Projection)]
        _lib.orc_render.argtypes = [C.POINTER(_Gaussians), C.POINTER(_Camera), C.POINTER(_Pose), _dp,
                                    C.c_int, _lp, C.c_int64, C.POINTER(_Images)]
        _lib.orc_render_alternatives.argtypes = [C.POINTER(_Gaussians), C.POINTER(_Camera), C.POINTER(_Pose),
                                                 _dp, C.c_int, _lp, C.c_int64, C.c_double, C.c_double, C.c_int32,
                                                 _dp, _ip]
        _lib.orc_backward.argtypes = [C.POINTER(_Gaussians), C.POINTER(_Camera), C.POINTER(_Pose), _dp,
                                      C.c_int, C.POINTER(_ImageGrads), C.POINTER(_Grads)]
        _lib.orc_fd_linear.argtypes = [C.POINTER(_Gaussians), C.POINTER(_Camera), C.POINTER(_Pose), _dp,
                                       C.POINTER(_ImageGrads), C.c_int64, _ip, _lp, _ip, C.c_double, _dp]
        _lib.orc_gaussian_uncertainty.argtypes = [C.POINTER(_Gaussians), C.POINTER(_Camera), C.POINTER(_Pose),
                                                  _dp, C.c_int, _dp, _lp, _ip, _dp]
        _lib.orc_sh_basis.argtypes = [C.c_int32, _dp, _dp, _dp]
        _lib.orc_sh_basis.restype = C.c_int
        _lib.orc_se3_exp.argtypes = [_dp, _dp, _dp]
        _lib.orc_se3_exp.restype = None
        _lib.orc_num_threads.restype = C.c_int
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


class _Scene:
    """Keeps the double copies alive while C holds their pointers.  A scene
    with an ``sh`` array [n, (degree + 1)^2, 3] takes its colour from it (the
    degree follows from its shape) and may omit ``rgb``."""

    def __init__(self, scene):
        sh = scene.get("sh")
        self.arrays = [_f64(scene[k]) for k in ("means", "log_scales", "quats", "opacity_logits")]
        self.arrays.append(None if scene.get("rgb") is None else _f64(scene["rgb"]))
        n = self.arrays[0].shape[0]
        self.degree = 0
        if sh is not None:
            sh = _f64(sh)
            K = sh.shape[1]
            self.degree = int(round(np.sqrt(K))) - 1
            if sh.shape != (n, (self.degree + 1) ** 2, 3):
                raise ValueError("sh must be [n, (degree + 1)^2, 3]")
        self.sh = sh
        self.c = _Gaussians(n, *[_ptr(a) for a in self.arrays], _ptr(sh), self.degree)
        self.n = n


def _cam(cam):
    return _Camera(int(cam["width"]), int(cam["height"]), float(cam["fx"]), float(cam["fy"]),
                   float(cam["cx"]), float(cam["cy"]))


def _pose(pose):
    R, t = pose
    p = _Pose()
    p.R[:] = [float(v) for v in np.asarray(R, dtype=np.float64).reshape(9)]
    p.t[:] = [float(v) for v in np.asarray(t, dtype=np.float64).reshape(3)]
    return p


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def project(scene, cam, pose) -> dict:
    """Per-Gaussian projection (Eq. 1-2) and the binning rectangle."""
    s = _Scene(scene)
    n = s.n
    out = dict(visible=np.zeros(n, np.int32), clamp=np.zeros((n, 2), np.int32),
               p_cam=np.zeros((n, 3)), mu=np.zeros((n, 2)), cov2d=np.zeros((n, 3)),
               conic=np.zeros((n, 3)), depth=np.zeros(n), opacity=np.zeros(n),
               rect=np.zeros((n, 4), np.int32), rect_edges=np.zeros((n, 4)))
    pr = _Projection(*[_ptr(out[k], _ip if out[k].dtype == np.int32 else _dp)
                       for k in ("visible", "clamp", "p_cam", "mu", "cov2d", "conic", "depth",
                                 "opacity", "rect", "rect_edges")])
    _check(lib().orc_project(C.byref(s.c), C.byref(_cam(cam)), C.byref(_pose(pose)), C.byref(pr)),
           "project")
    return out


def render(scene, cam, pose, depth_obs=None, *, candidates: int = 1, pixels=None) -> dict:
    """Render colour [3,H,W], depth, opacity, median depth and uncertainty.

    ``pixels`` (flat indices v*W+u) renders only those pixels; then every map
    is flat over them.  ``candidates=0`` is the brute-force walk over every
    visible Gaussian, ``1`` restricts it to the Gaussians whose binning
    rectangle holds the pixel (same result)."""
    s = _Scene(scene)
    H, W = int(cam["height"]), int(cam["width"])
    if pixels is None:
        shape2, px, npx = (H, W), None, H * W
    else:
        px = np.ascontiguousarray(np.asarray(pixels, dtype=np.int64).reshape(-1))
        shape2, npx = (px.size,), px.size
    d = None if depth_obs is None else _f64(depth_obs)
    out = dict(color=np.zeros((3,) + shape2), depth=np.zeros(shape2), opacity=np.zeros(shape2),
               depth_median=np.zeros(shape2), uncertainty=np.zeros(shape2),
               n_contrib=np.zeros(shape2, np.int32), t_final=np.zeros(shape2),
               median_id=np.zeros(shape2, np.int32), decision_margin=np.zeros(shape2),
               order_margin=np.zeros(shape2), stop_order_margin=np.zeros(shape2))
    im = _Images(*[_ptr(out[k], _ip if out[k].dtype == np.int32 else _dp)
                   for k in ("color", "depth", "opacity", "depth_median", "uncertainty",
                             "n_contrib", "t_final", "median_id", "decision_margin", "order_margin",
                             "stop_order_margin")])
    _check(lib().orc_render(C.byref(s.c), C.byref(_cam(cam)), C.byref(_pose(pose)), _ptr(d),
                            int(candidates), _ptr(px, _lp), int(npx), C.byref(im)), "render")
    if depth_obs is None:
        out["uncertainty"] = None
    return out


#: Values of one alternative result of render_alternatives, in order.
ALT_VALUES = ("color_r", "color_g", "color_b", "depth", "opacity", "depth_median", "uncertainty", "t_final")


def render_alternatives(scene, cam, pose, depth_obs, pixels, decision_margin, order_margin, *,
                        max_alts: int = 64, candidates: int = 1):
    """Every admissible result of the listed pixels (flat indices v*W+u) when
    the decisions of Eq. 3-5 and 7-8 that sit within ``decision_margin``
    (relative) of their thresholds, and the order of Gaussians whose depths
    differ by less than ``order_margin`` (relative), may go either way (see
    orc_render_alternatives).  Returns (alts [n, max_alts, 8] in the order of
    ALT_VALUES, count [n]); count > max_alts means more than max_alts."""
    s = _Scene(scene)
    px = np.ascontiguousarray(np.asarray(pixels, dtype=np.int64).reshape(-1))
    d = None if depth_obs is None else _f64(depth_obs)
    alts = np.zeros((px.size, int(max_alts), len(ALT_VALUES)))
    count = np.zeros(px.size, np.int32)
    _check(lib().orc_render_alternatives(C.byref(s.c), C.byref(_cam(cam)), C.byref(_pose(pose)), _ptr(d),
                                         int(candidates), _ptr(px, _lp), int(px.size), float(decision_margin),
                                         float(order_margin), int(max_alts), _ptr(alts), _ptr(count, _ip)),
           "render_alternatives")
    return alts, count


def _image_grads(dimg):
    keep = {}
    for k in ("color", "depth", "opacity", "depth_median", "uncertainty"):
        v = None if dimg is None else dimg.get(k)
        keep[k] = None if v is None else _f64(v)
    return keep, _ImageGrads(*[_ptr(keep[k]) for k in ("color", "depth", "opacity", "depth_median",
                                                        "uncertainty")])


def backward(scene, cam, pose, depth_obs, dimg: dict, *, candidates: int = 1) -> dict:
    """Analytic gradient of sum(dimg * maps) w.r.t. every parameter and the pose.

    ``pose`` gradient is the left se(3) perturbation (rho, phi) of the
    world->camera transform.  Also returns the gradients with respect to the
    projected quantities (``proj_mu``, ``proj_conic``, ``proj_opacity``,
    ``proj_depth``)."""
    s = _Scene(scene)
    n = s.n
    keep, ig = _image_grads(dimg)
    d = None if depth_obs is None else _f64(depth_obs)
    out = dict(means=np.zeros((n, 3)), log_scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
               opacity_logits=np.zeros(n), rgb=np.zeros((n, 3)), pose=np.zeros(6),
               sh=None if s.sh is None else np.zeros(s.sh.shape),
               proj_mu=np.zeros((n, 2)), proj_conic=np.zeros((n, 3)), proj_opacity=np.zeros(n),
               proj_depth=np.zeros(n))
    gr = _Grads(*[_ptr(out[k]) for k in ("means", "log_scales", "quats", "opacity_logits", "rgb",
                                          "pose", "sh", "proj_mu", "proj_conic", "proj_opacity",
                                          "proj_depth")])
    _check(lib().orc_backward(C.byref(s.c), C.byref(_cam(cam)), C.byref(_pose(pose)), _ptr(d),
                              int(candidates), C.byref(ig), C.byref(gr)), "backward")
    return out


PARAM_KINDS = {"means": 0, "log_scales": 1, "quats": 2, "opacity_logits": 3, "rgb": 4, "pose": 5, "sh": 6}


def fd_linear(scene, cam, pose, depth_obs, dimg: dict, coords, rel_step: float = 1e-6) -> np.ndarray:
    """Frozen-decision central differences of sum(dimg * maps).

    ``coords`` is a list of ``(kind, index, component)`` with kind one of
    ``PARAM_KINDS``; for ``"pose"`` the component is the xi coordinate
    (rho then phi) and the index is ignored; for ``"sh"`` it is 3 k + c."""
    s = _Scene(scene)
    keep, ig = _image_grads(dimg)
    d = None if depth_obs is None else _f64(depth_obs)
    kinds = np.array([PARAM_KINDS[c[0]] for c in coords], np.int32)
    idx = np.array([int(c[1]) for c in coords], np.int64)
    comp = np.array([int(c[2]) for c in coords], np.int32)
    out = np.zeros(len(coords))
    _check(lib().orc_fd_linear(C.byref(s.c), C.byref(_cam(cam)), C.byref(_pose(pose)), _ptr(d),
                               C.byref(ig), len(coords), _ptr(kinds, _ip), _ptr(idx, _lp),
                               _ptr(comp, _ip), float(rel_step), _ptr(out)), "fd_linear")
    return out


#: Pruning threshold on the per-Gaussian uncertainty (Sec. 3.2).
NU_TAU = 0.025
#: Opacity a pruned Gaussian is lowered to (the paper says only "a low-opacity
#: level"; reading: 0.01).
NU_LOW_OPACITY = 0.01


def gaussian_uncertainty(scene, cam, pose, depth_obs, nu_sum=None, nu_count=None, *, candidates: int = 1):
    """One keyframe's contribution to Eq. 13 (see orc_gaussian_uncertainty).

    nu_sum / nu_count: running float64 [n] / int64 [n] accumulators (new
    zeros if None), updated in place.  Returns dict(sum, count, dominant
    [H, W] int32, margin [H, W])."""
    s = _Scene(scene)
    n = s.n
    nu_sum = np.zeros(n) if nu_sum is None else nu_sum
    nu_count = np.zeros(n, np.int64) if nu_count is None else nu_count
    assert nu_sum.dtype == np.float64 and nu_count.dtype == np.int64
    H, W = int(cam["height"]), int(cam["width"])
    dom = np.zeros((H, W), np.int32)
    margin = np.zeros((H, W))
    d = _f64(depth_obs)
    _check(lib().orc_gaussian_uncertainty(C.byref(s.c), C.byref(_cam(cam)), C.byref(_pose(pose)), _ptr(d),
                                          int(candidates), _ptr(nu_sum), _ptr(nu_count, _lp), _ptr(dom, _ip),
                                          _ptr(margin)), "gaussian_uncertainty")
    return dict(sum=nu_sum, count=nu_count, dominant=dom, margin=margin)


def nu_from_sums(nu_sum, nu_count):
    """Eq. 13: nu_i = (sum over dominated pixels of the window) / (M_1 + ... + M_k);
    a Gaussian that dominates no pixel has no evidence and gets nu = 0."""
    nu_sum = np.asarray(nu_sum, np.float64)
    nu_count = np.asarray(nu_count)
    out = np.zeros_like(nu_sum)
    has = nu_count > 0
    out[has] = nu_sum[has] / nu_count[has]
    return out


def prune_uncertain(opacity_logits, nu, tau=NU_TAU, level=NU_LOW_OPACITY):
    """Sec. 3.2: Gaussians with nu > tau have their opacity lowered to `level`
    (never raised).  Returns (new opacity logits, boolean mask of pruned)."""
    o = np.asarray(opacity_logits, np.float64).copy()
    mask = np.asarray(nu) > tau
    cap = np.log(level / (1.0 - level))
    o[mask] = np.minimum(o[mask], cap)
    return o, mask


def sh_basis(degree: int, d):
    """Real spherical harmonics of the colour reading (orc_sh_basis) at unit
    direction d: returns (Y [K], dY [K, 3])."""
    K = (int(degree) + 1) ** 2
    Y, dY = np.zeros(K), np.zeros((K, 3))
    dd = _f64(np.asarray(d).reshape(3))
    if lib().orc_sh_basis(int(degree), _ptr(dd), _ptr(Y), _ptr(dY)) != K:
        raise ValueError("degree must be 0 .. 3")
    return Y, dY


def se3_exp(xi):
    """SE(3) exponential of xi = (rho, phi) -> (R[3,3], t[3])."""
    x = _f64(xi).reshape(6)
    R = np.zeros(9)
    t = np.zeros(3)
    lib().orc_se3_exp(_ptr(x), _ptr(R), _ptr(t))
    return R.reshape(3, 3), t


def retract(pose, xi):
    """Left retraction used by tracking: T <- exp(xi^) T."""
    dR, dt = se3_exp(xi)
    R, t = (np.asarray(a, dtype=np.float64) for a in pose)
    return dR @ R, dR @ t + dt


# --------------------------------------------------------------------------
# Losses (Eq. 14, 16, 19) and their gradient images
# --------------------------------------------------------------------------

def l1_color_loss(color, target):
    """Eq. 14: mean over the H*W pixels of the L1 norm over the 3 channels."""
    hw = color.shape[-1] * color.shape[-2]
    diff = np.asarray(color, np.float64) - np.asarray(target, np.float64)
    return np.abs(diff).sum() / hw, np.sign(diff) / hw


def l1_depth_loss(depth, target):
    """Eq. 16: mean absolute difference of the alpha-blended and observed depth."""
    hw = depth.shape[-1] * depth.shape[-2]
    diff = np.asarray(depth, np.float64) - np.asarray(target, np.float64)
    return np.abs(diff).sum() / hw, np.sign(diff) / hw


def tracking_loss(maps, target_color, target_depth, lam=(0.2, 1.0)):
    """Eq. 19: lambda1 * L_color + lambda2 * L_geo; returns (loss, dimg)."""
    lc, gc = l1_color_loss(maps["color"], target_color)
    ld, gd = l1_depth_loss(maps["depth"], target_depth)
    return lam[0] * lc + lam[1] * ld, dict(color=lam[0] * gc, depth=lam[1] * gd)


def uncertainty_weighted_loss(maps, target_color, target_depth):
    """Mapping loss of the 1200x680 workload: L1 colour (Eq. 14) plus the L1
    depth error (Eq. 16) weighted per pixel by the rendered uncertainty U
    (Eq. 10); the gradient flows through both factors."""
    lc, gc = l1_color_loss(maps["color"], target_color)
    hw = maps["depth"].shape[-1] * maps["depth"].shape[-2]
    diff = np.asarray(maps["depth"], np.float64) - np.asarray(target_depth, np.float64)
    U = np.asarray(maps["uncertainty"], np.float64)
    loss = lc + (U * np.abs(diff)).sum() / hw
    return loss, dict(color=gc, depth=U * np.sign(diff) / hw, uncertainty=np.abs(diff) / hw)


def adam_step(param, grad, m, v, step, lr, betas=(0.9, 0.999), eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1) with bias correction.
    ``step`` counts from 1.  Returns (new_param, m, v)."""
    b1, b2 = betas
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return param - lr * mhat / (np.sqrt(vhat) + eps), m, v


def tile_lists(proj, cam, tile: int = 16):
    """Tile binning by its definition: tile (tx, ty) holds every visible
    Gaussian whose binning rectangle overlaps it, ordered by (depth, index).
    Returns {tile_index: np.ndarray of Gaussian ids}."""
    tiles_x = (int(cam["width"]) + tile - 1) // tile
    vis = np.nonzero(proj["visible"])[0]
    order = vis[np.lexsort((vis, proj["depth"][vis]))]
    lists = {}
    for i in order:
        u0, u1, v0, v1 = (int(v) for v in proj["rect"][i])
        for ty in range(v0 // tile, v1 // tile + 1):
            for tx in range(u0 // tile, u1 // tile + 1):
                lists.setdefault(ty * tiles_x + tx, []).append(int(i))
    return {k: np.array(v, np.int64) for k, v in lists.items()}
