"""PyTorch-facing wrappers of the cgsr C ABI.

PyTorch supplies device memory and streams; every step of rendering, its
backward, the tracking loss gradient and the pose update runs in the HIP
kernels of ``libcgsr.so``.  Functions here allocate output tensors, check
shapes and dtypes, and pass raw pointers through :mod:`binding`.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import binding as B

MAP_NAMES = ("color", "depth", "opacity", "depth_median", "uncertainty")
PARAM_NAMES = ("means", "log_scales", "quats", "opacity_logits", "rgb")
PARAM_WIDTH = {"means": 3, "log_scales": 3, "quats": 4, "opacity_logits": 1, "rgb": 3}

#: Learning rates of sequential tracking, rotation (so(3)) and translation
#: parts (Sec. 4, Implementation Details).
TRACK_LR_PHI = 0.0015
TRACK_LR_RHO = 0.00215
#: Replica weights of the tracking loss, Eq. 19 (Sec. 4).
TRACK_LAMBDA = (0.2, 1.0)


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _check_f32(name, t, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def sh_degree_of(sh: torch.Tensor) -> int:
    """Degree of an SH coefficient tensor [n, (degree + 1)^2, 3]."""
    K = sh.shape[1] if sh.dim() == 3 else -1
    for d in range(4):
        if K == (d + 1) ** 2 and sh.shape[2] == 3:
            return d
    raise ValueError("sh must be [n, (degree + 1)^2, 3] with degree 0 .. 3")


def gaussians_struct(scene: dict) -> B.cgsr_gaussians:
    """Parameters of ``scene``; with an ``sh`` tensor [n, (degree + 1)^2, 3]
    the colour is view-dependent and ``rgb`` may be absent."""
    n = scene["means"].shape[0]
    sh = scene.get("sh")
    for k in PARAM_NAMES:
        if k == "rgb" and sh is not None and scene.get("rgb") is None:
            continue
        w = PARAM_WIDTH[k]
        _check_f32(k, scene[k], (n,) if w == 1 else (n, w))
    deg = 0
    if sh is not None:
        deg = sh_degree_of(sh)
        _check_f32("sh", sh, (n, (deg + 1) ** 2, 3))
    return B.cgsr_gaussians(n, *[_ptr(scene.get(k)) for k in PARAM_NAMES], _ptr(sh), deg)


def camera_struct(cam: dict) -> B.cgsr_camera:
    return B.cgsr_camera(int(cam["width"]), int(cam["height"]), float(cam["fx"]), float(cam["fy"]),
                         float(cam["cx"]), float(cam["cy"]))


def pose_tensor(R, t, device="cuda") -> torch.Tensor:
    """Pack a world->camera pose into the float32[12] layout of the ABI."""
    R = torch.as_tensor(R, dtype=torch.float64).reshape(9)
    t = torch.as_tensor(t, dtype=torch.float64).reshape(3)
    return torch.cat([R, t]).to(torch.float32).to(device).contiguous()


class State:
    """Owns one cgsr_state (the workspace of a render and its backward)."""

    def __init__(self, sync_capacity: bool = True, timing: bool = False, fwd_ppl: int | None = None,
                 bwd_ppl: int | None = None, count_work: bool = True):
        s = B.cgsr_default_settings()
        s.sync_capacity = int(sync_capacity)
        s.timing = int(timing)
        s.count_work = int(count_work)
        if fwd_ppl is not None:
            s.fwd_pixels_per_lane = int(fwd_ppl)
        if bwd_ppl is not None:
            s.bwd_pixels_per_lane = int(bwd_ppl)
        self.settings = s
        self.handle = B.cgsr_state_create(s)
        self.n_views = 0
        self.n = 0

    def reserve(self, records=0, pixels=0, tiles=0, tile_pairs=0):
        """Grow the workspace; tile_pairs: (tile, Gaussian) pairs one tile's
        bucket holds (size it from ``stats().peak_pairs``)."""
        B.cgsr_state_reserve(self.handle, int(records), int(pixels), int(tiles), int(tile_pairs))

    def stats(self) -> B.cgsr_stats:
        return B.cgsr_get_stats(self.handle, _stream())

    def check(self):
        B.cgsr_state_check(self.handle, _stream())

    def time_tracking_blend(self, reps: int = 200) -> float:
        """Average ms of one launch of the last tracking step's fused blend
        kernel, over ``reps`` back-to-back re-runs between two HIP events."""
        return B.cgsr_time_tracking_blend(self.handle, int(reps), _stream())

    def timings(self) -> dict:
        return B.cgsr_get_timings(self.handle)

    def close(self):
        if self.handle:
            B.cgsr_state_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def render(state: State, scene: dict, poses: torch.Tensor, cams, depth_obs=None,
           maps=MAP_NAMES) -> list:
    """Render ``len(cams)`` views in one launch sequence.

    poses: float32 CUDA tensor [V, 12] (or [12] for one view).  depth_obs:
    None or a list of [H, W] tensors (None entries allowed).  Returns one dict
    of maps per view (only those in ``maps``; ``uncertainty`` needs depth)."""
    if isinstance(cams, dict):
        cams = [cams]
    V = len(cams)
    poses = poses.reshape(V, 12)
    _check_f32("poses", poses)
    g = gaussians_struct(scene)
    dev = poses.device
    outs, structs, deps = [], [], []
    for v, cam in enumerate(cams):
        H, W = int(cam["height"]), int(cam["width"])
        d = None if depth_obs is None else depth_obs[v]
        if d is not None:
            _check_f32(f"depth_obs[{v}]", d, (H, W))
        o = {}
        for k in maps:
            if k == "uncertainty" and d is None:
                continue
            o[k] = torch.empty((3, H, W) if k == "color" else (H, W), dtype=torch.float32, device=dev)
        outs.append(o)
        structs.append(B.cgsr_images(*[_ptr(o.get(k)) for k in MAP_NAMES]))
        deps.append(_ptr(d))
    B.cgsr_render(state.handle, g, V, poses.data_ptr(), [camera_struct(c) for c in cams],
                  None if depth_obs is None else deps, structs, _stream())
    state.n_views, state.n = V, g.n
    state.sh_shape = None if scene.get("sh") is None else tuple(scene["sh"].shape)
    # The backward reads these through the pointers the state recorded.
    state.inputs = (scene, poses, depth_obs)
    return outs


#: Pruning threshold on the per-Gaussian uncertainty (Sec. 3.2).
NU_TAU = 0.025
#: Opacity a pruned Gaussian is lowered to (reading of "a low-opacity level").
NU_LOW_OPACITY = 0.01


def render_nu(state: State, scene: dict, poses: torch.Tensor, cams, depth_obs, nu_sum: torch.Tensor,
              nu_count: torch.Tensor, maps=MAP_NAMES, dominant: bool = False):
    """Render like ``render`` and accumulate the per-Gaussian uncertainty sums
    of Eq. 13 into nu_sum (float32 [n]) and nu_count (int32 [n], read as
    uint32 by the library).  Returns (list of map dicts, list of int32 [H, W]
    dominant-Gaussian maps or None)."""
    if isinstance(cams, dict):
        cams = [cams]
    V = len(cams)
    poses = poses.reshape(V, 12)
    _check_f32("poses", poses)
    g = gaussians_struct(scene)
    n = g.n
    _check_f32("nu_sum", nu_sum, (n,))
    if not (isinstance(nu_count, torch.Tensor) and nu_count.is_cuda and nu_count.dtype == torch.int32
            and nu_count.is_contiguous() and tuple(nu_count.shape) == (n,)):
        raise ValueError("nu_count must be a contiguous int32 CUDA tensor of shape [n]")
    dev = poses.device
    outs, structs, doms = [], [], []
    for v, cam in enumerate(cams):
        H, W = int(cam["height"]), int(cam["width"])
        _check_f32(f"depth_obs[{v}]", depth_obs[v], (H, W))
        o = {k: torch.empty((3, H, W) if k == "color" else (H, W), dtype=torch.float32, device=dev) for k in maps}
        outs.append(o)
        structs.append(B.cgsr_images(*[_ptr(o.get(k)) for k in MAP_NAMES]))
        doms.append(torch.empty((H, W), dtype=torch.int32, device=dev) if dominant else None)
    B.cgsr_render_nu(state.handle, g, V, poses.data_ptr(), [camera_struct(c) for c in cams],
                     [d.data_ptr() for d in depth_obs], structs, [_ptr(d) for d in doms] if dominant else None,
                     nu_sum.data_ptr(), nu_count.data_ptr(), _stream())
    state.n_views, state.n = V, n
    state.sh_shape = None if scene.get("sh") is None else tuple(scene["sh"].shape)
    state.inputs = (scene, poses, depth_obs)
    return outs, (doms if dominant else None)


#: Rendered-opacity threshold of Gaussian spawning (Sec. 3.3).
SPAWN_PSI = 0.5
GAUSSIAN_ARRAYS = ("means", "log_scales", "quats", "opacity_logits", "rgb", "sh")


def arrays_struct(params: dict) -> B.cgsr_gaussian_arrays:
    """Writable arrays of a Gaussian set (rows beyond the count are spare
    capacity); ``sh`` [rows, K, 3] replaces ``rgb`` for view-dependent colour."""
    for k in GAUSSIAN_ARRAYS:
        if params.get(k) is not None:
            _check_f32(k, params[k])
    sh = params.get("sh")
    return B.cgsr_gaussian_arrays(*[_ptr(params.get(k)) for k in GAUSSIAN_ARRAYS],
                                  0 if sh is None else sh_degree_of(sh))


def empty_like_set(params: dict, rows: int) -> dict:
    """Uninitialised arrays of the same layout with ``rows`` Gaussians."""
    return {k: torch.empty((rows,) + tuple(v.shape[1:]), dtype=torch.float32, device=v.device)
            for k, v in params.items() if k in GAUSSIAN_ARRAYS and v is not None}


def spawn_gaussians(params: dict, n: int, cam: dict, pose: torch.Tensor, color: torch.Tensor, depth: torch.Tensor,
                    opacity: torch.Tensor | None = None, psi: float = SPAWN_PSI, stride: int = 1,
                    init_logit: float = 0.0) -> int:
    """Sec. 3.3 spawning into ``params`` (arrays with spare rows, n in use)
    from the pixels of one RGB-D view whose rendered opacity is below psi (all
    pixels with a depth when ``opacity`` is None).  Returns the new count."""
    capacity = params["means"].shape[0]
    H, W = int(cam["height"]), int(cam["width"])
    _check_f32("color", color, (3, H, W))
    _check_f32("depth", depth, (H, W))
    if opacity is not None:
        _check_f32("opacity", opacity, (H, W))
    return B.cgsr_spawn_gaussians(arrays_struct(params), int(n), int(capacity), camera_struct(cam),
                                  pose.reshape(12).data_ptr(), color.data_ptr(), depth.data_ptr(), _ptr(opacity),
                                  float(psi), int(stride), float(init_logit), _stream())


def compact_gaussians(params: dict, keep: torch.Tensor, extra=(), no_alloc: bool = False):
    """The Gaussians with keep != 0 (uint8 [n]) in order: returns (new arrays
    trimmed to the kept count, list of compacted extra tensors).  ``extra``:
    per-Gaussian float32 tensors [n, ...] compacted alike.  no_alloc: the
    library call uses its fixed per-GPU scratch instead of allocating (n up to
    CGSR_COMPACT_NOALLOC_MAX_N); the output tensors are still allocated here."""
    n = params["means"].shape[0]
    if not (keep.is_cuda and keep.dtype == torch.uint8 and keep.numel() == n and keep.is_contiguous()):
        raise ValueError("keep must be a contiguous uint8 CUDA tensor of n entries")
    dst = empty_like_set(params, n)
    ex_dst = [torch.empty_like(e) for e in extra]
    widths = [int(e.numel() // max(n, 1)) for e in extra]
    fn = B.cgsr_compact_gaussians_noalloc if no_alloc else B.cgsr_compact_gaussians
    m = fn(n, keep.data_ptr(), arrays_struct(params), arrays_struct(dst), [e.data_ptr() for e in extra],
           [e.data_ptr() for e in ex_dst], widths, _stream())
    return {k: v[:m] for k, v in dst.items()}, [e[:m] for e in ex_dst]


def set_densify_stats(state: State, grad_accum: torch.Tensor | None, count: torch.Tensor | None):
    """Accumulate |dL/dmu| and visibility counts of every later backward on
    ``state`` (float32 [n], int32 [n] read as uint32); None stops."""
    B.cgsr_set_densify_stats(state.handle, _ptr(grad_accum), _ptr(count))


def densify_gaussians(params: dict, grad_accum: torch.Tensor, count: torch.Tensor, grad_threshold: float,
                      dense_scale: float, normals: torch.Tensor):
    """Clone / split densification (Sec. 3.3, kept from splatting); normals:
    float32 [n, 2, 3] standard normal draws.  Returns the new arrays."""
    n = params["means"].shape[0]
    _check_f32("grad_accum", grad_accum, (n,))
    _check_f32("normals", normals, (n, 2, 3))
    dst = empty_like_set(params, max(2 * n, 1))
    m = B.cgsr_densify_gaussians(n, grad_accum.data_ptr(), count.data_ptr(), float(grad_threshold),
                                 float(dense_scale), normals.data_ptr(), arrays_struct(params), arrays_struct(dst),
                                 max(2 * n, 1), _stream())
    return {k: v[:m] for k, v in dst.items()}


def nu_prune(nu_sum: torch.Tensor, nu_count: torch.Tensor, tau: float = NU_TAU, low_opacity: float = NU_LOW_OPACITY,
             opacity_logits: torch.Tensor | None = None):
    """nu of Eq. 13 from the window's sums and the tau rule of Sec. 3.2 applied
    in place to opacity_logits (if given).  Returns (nu [n], pruned count
    as a 1-element int32 device tensor)."""
    n = nu_sum.shape[0]
    nu = torch.empty_like(nu_sum)
    cnt = torch.zeros(1, dtype=torch.int32, device=nu_sum.device)
    B.cgsr_nu_prune(n, nu_sum.data_ptr(), nu_count.data_ptr(), float(tau), float(low_opacity), _ptr(opacity_logits),
                    nu.data_ptr(), cnt.data_ptr(), _stream())
    return nu, cnt


#: Eq. 18 weights (colour, ssim, geo, align, iso, var), Sec. 4.
MAPPING_OMEGA_REPLICA = (0.7, 0.1, 0.25, 0.25, 0.1, 0.15)
MAPPING_OMEGA_TUM_SCANNET = (1.0, 0.1, 0.8, 0.5, 0.1, 0.5)
#: Eq. 17 anisotropy level (Sec. 3.3).
ISO_EPSILON = 1.0


def mapping_objective(state: State, maps, target_colors, target_depths, omega=MAPPING_OMEGA_REPLICA,
                      iso_epsilon: float = ISO_EPSILON, dlog_scales: torch.Tensor | None = None,
                      loss: torch.Tensor | None = None):
    """Gradient images of Eq. 18 for the views of the last render on ``state``.

    maps: list (one per view) of dicts with the rendered colour, depth,
    depth_median and uncertainty the weighted terms need.  Returns a list of
    dicts of gradient images (colour, depth, depth_median, uncertainty, as
    the weights need them) to hand to ``backward``; the isotropy gradient is
    added into dlog_scales ([n, 3]) and the per-view objective into loss
    ([V]) when given."""
    w = B.cgsr_mapping_weights(*[float(x) for x in omega], float(iso_epsilon))
    V = len(maps)
    if V != state.n_views:
        raise ValueError(f"expected {state.n_views} views of maps, got {V}")
    outs, m_s, d_s = [], [], []
    for m in maps:
        d = {}
        if omega[0] != 0 or omega[1] != 0:
            d["color"] = torch.empty_like(m["color"])
        if omega[2] != 0 or omega[3] != 0:
            d["depth"] = torch.empty_like(m["depth"])
        if omega[3] != 0:
            d["depth_median"] = torch.empty_like(m["depth"])
        if omega[5] != 0:
            d["uncertainty"] = torch.empty_like(m["depth"])
        outs.append(d)
        m_s.append(B.cgsr_images(*[_ptr(m.get(k)) for k in MAP_NAMES]))
        d_s.append(B.cgsr_images(*[_ptr(d.get(k)) for k in MAP_NAMES]))
    B.cgsr_mapping_objective(state.handle, w, m_s, [_ptr(t) for t in target_colors] if target_colors else None,
                             [_ptr(t) for t in target_depths] if target_depths else None, d_s, _ptr(dlog_scales),
                             _ptr(loss), _stream())
    return outs


#: Mapping learning rates (reading: the paper defers them to its supplementary
#: material; these are the 3D Gaussian splatting defaults, the position rate
#: scaled by a 5 m scene extent).
MAPPING_LR = dict(means=1.6e-4 * 5.0, log_scales=5e-3, quats=1e-3, opacity_logits=5e-2, rgb=2.5e-3,
                  sh_rest=2.5e-3 / 20.0)


def gaussian_adam_params(lr=None, betas=(0.9, 0.999), eps=1e-15, sh_degree: int = 0) -> B.cgsr_gaussian_adam_params:
    """Adam constants; with SH colour, lr["rgb"] is the rate of the degree-0
    coefficients and lr["sh_rest"] that of the others."""
    lr = dict(MAPPING_LR, **(lr or {}))
    return B.cgsr_gaussian_adam_params(*[float(lr[k]) for k in PARAM_NAMES], float(betas[0]), float(betas[1]),
                                       float(eps), float(lr["sh_rest"]), int(sh_degree))


def gaussian_grads_struct(tensors: dict) -> B.cgsr_gaussian_grads:
    """Pointers of a parameter or gradient dict; ``sh`` replaces ``rgb`` for
    view-dependent colour."""
    n = tensors["means"].shape[0]
    sh = tensors.get("sh")
    for k in PARAM_NAMES:
        if k == "rgb" and sh is not None and tensors.get("rgb") is None:
            continue
        w = PARAM_WIDTH[k]
        _check_f32(k, tensors[k], (n,) if w == 1 else (n, w))
    if sh is not None:
        _check_f32("sh", sh, (n, sh.shape[1], 3))
    return B.cgsr_gaussian_grads(*[_ptr(tensors.get(k)) for k in PARAM_NAMES], _ptr(sh))


def gaussian_adam_step(scene: dict, grads: dict, moments: torch.Tensor, step: torch.Tensor, lr=None,
                       betas=(0.9, 0.999), eps=1e-15):
    """In-place Adam step on every Gaussian parameter tensor of ``scene`` with
    ``grads`` (zeroed afterwards).  moments: float32 [2, (11 + W) n] zeros,
    W = 3 for rgb or 3 (degree + 1)^2 for SH colour; step: int32 [1] zeros
    (read as uint32 by the library)."""
    n = scene["means"].shape[0]
    sh = scene.get("sh")
    deg = 0 if sh is None else sh_degree_of(sh)
    W = 3 if sh is None else 3 * (deg + 1) ** 2
    _check_f32("moments", moments, (2, (11 + W) * n))
    g_struct = gaussian_grads_struct(scene)
    if sh is not None:
        g_struct.rgb = None
    d_struct = gaussian_grads_struct(grads)
    if sh is not None:
        d_struct.rgb = None
    B.cgsr_gaussian_adam_step(n, g_struct, d_struct, moments.data_ptr(), step.data_ptr(),
                              gaussian_adam_params(lr, betas, eps, deg), _stream())


class BundleAdjuster:
    """Sliding-window bundle adjustment (Sec. 3.4, Eq. 21) over k keyframes:
    one iteration renders every keyframe in one launch sequence (with its
    sensor depth, for the uncertainty terms), forms the gradient images of
    the mapping objective (Eq. 18), back-propagates to the Gaussians and to
    each keyframe pose, then takes an Adam step on the Gaussians and one on
    the poses.  All buffers are allocated once, so ``step`` can be captured
    into a HIP graph after one eager call has sized the workspace."""

    def __init__(self, scene: dict, poses: torch.Tensor, cams, target_colors, target_depths,
                 omega=MAPPING_OMEGA_REPLICA, lr=None, pose_lr=(TRACK_LR_RHO, TRACK_LR_PHI), optimize_poses=True,
                 eps=1e-15):
        self.scene, self.cams = scene, list(cams)
        V = len(self.cams)
        self.poses = poses.reshape(V, 12)
        _check_f32("poses", self.poses)
        self.tc, self.td = list(target_colors), list(target_depths)
        self.omega = tuple(omega)
        n = scene["means"].shape[0]
        dev = self.poses.device
        sh = scene.get("sh")
        self.sh_degree = 0 if sh is None else sh_degree_of(sh)
        names = [k for k in PARAM_NAMES if not (k == "rgb" and sh is not None)] + (["sh"] if sh is not None else [])
        self.grads = {k: torch.zeros_like(scene[k]) for k in names}
        W = 3 if sh is None else 3 * (self.sh_degree + 1) ** 2
        self.moments = torch.zeros((2, (11 + W) * n), dtype=torch.float32, device=dev)
        self.step_count = torch.zeros(1, dtype=torch.int32, device=dev)
        self.dposes = torch.zeros((V, 6), dtype=torch.float32, device=dev)
        self.pose_adam = torch.zeros((V, 16), dtype=torch.float32, device=dev)
        self.loss = torch.zeros(V, dtype=torch.float32, device=dev)
        self.state = State(sync_capacity=True)
        self.g = gaussians_struct(scene)
        self.cam_s = [camera_struct(c) for c in self.cams]
        self.maps = []
        for c in self.cams:
            H, W = int(c["height"]), int(c["width"])
            self.maps.append(dict(color=torch.empty((3, H, W), device=dev), depth=torch.empty((H, W), device=dev),
                                  depth_median=torch.empty((H, W), device=dev),
                                  uncertainty=torch.empty((H, W), device=dev)))
        self.dimgs = [{k: torch.empty_like(m[k]) for k in m} for m in self.maps]
        self.map_s = [B.cgsr_images(*[_ptr(m.get(k)) for k in MAP_NAMES]) for m in self.maps]
        self.dimg_s = [B.cgsr_images(*[_ptr(d.get(k)) for k in MAP_NAMES]) for d in self.dimgs]
        self.weights = B.cgsr_mapping_weights(*[float(x) for x in self.omega], float(ISO_EPSILON))
        self.hp = gaussian_adam_params(lr, eps=eps, sh_degree=self.sh_degree)
        self.pose_hp = adam_params(pose_lr[0], pose_lr[1])
        self.param_s = gaussian_grads_struct(scene)
        self.grad_s = gaussian_grads_struct(self.grads)
        self.optimize_poses = optimize_poses

    def step(self):
        s = _stream()
        V = len(self.cams)
        st = self.state.handle
        B.cgsr_render(st, self.g, V, self.poses.data_ptr(), self.cam_s, [t.data_ptr() for t in self.td], self.map_s, s)
        B.cgsr_mapping_objective(st, self.weights, self.map_s, [t.data_ptr() for t in self.tc],
                                 [t.data_ptr() for t in self.td], self.dimg_s, self.grads["log_scales"].data_ptr(),
                                 self.loss.data_ptr(), s)
        B.cgsr_backward(st, self.dimg_s, self.grad_s, self.dposes.data_ptr() if self.optimize_poses else None, s)
        B.cgsr_gaussian_adam_step(self.scene["means"].shape[0], self.param_s, self.grad_s, self.moments.data_ptr(),
                                  self.step_count.data_ptr(), self.hp, s)
        if self.optimize_poses:
            B.cgsr_pose_adam_step(V, self.poses.data_ptr(), self.dposes.data_ptr(), self.pose_adam.data_ptr(),
                                  self.pose_hp, s)

    def check(self):
        self.state.check()


def backward(state: State, dimgs, param_grads: bool = True, pose_grads: bool = True):
    """Backward of the last render on ``state``.

    dimgs: list (one per view) of dicts of upstream gradient maps (missing =
    zero).  Returns (dict of parameter gradients or None, dposes [V,6] or None)."""
    V, n = state.n_views, state.n
    if len(dimgs) != V:
        raise ValueError(f"expected {V} gradient dicts, got {len(dimgs)}")
    keep, structs = [], []
    for d in dimgs:
        dd = {k: (None if d.get(k) is None else d[k].contiguous().float()) for k in MAP_NAMES}
        keep.append(dd)
        structs.append(B.cgsr_images(*[_ptr(dd[k]) for k in MAP_NAMES]))
    dev = next((t.device for d in keep for t in d.values() if t is not None), torch.device("cuda"))
    grads = None
    dG = None
    if param_grads:
        sh_shape = getattr(state, "sh_shape", None)
        names = [k for k in PARAM_NAMES if not (k == "rgb" and sh_shape is not None)]
        grads = {k: torch.zeros((n,) if PARAM_WIDTH[k] == 1 else (n, PARAM_WIDTH[k]), dtype=torch.float32,
                                device=dev) for k in names}
        if sh_shape is not None:
            grads["sh"] = torch.zeros(sh_shape, dtype=torch.float32, device=dev)
        dG = gaussian_grads_struct(grads)
    dposes = torch.zeros((V, 6), dtype=torch.float32, device=dev) if pose_grads else None
    B.cgsr_backward(state.handle, structs, dG, _ptr(dposes), _stream())
    return grads, dposes


def tracking_loss_grad(color, depth, target_color, target_depth, lam=TRACK_LAMBDA, dcolor=None, ddepth=None,
                       loss=None):
    """Gradient images of Eq. 19 (lambda1 * L_color + lambda2 * L_geo) on the device."""
    H, W = depth.shape
    dcolor = torch.empty_like(color) if dcolor is None else dcolor
    ddepth = torch.empty_like(depth) if ddepth is None else ddepth
    B.cgsr_tracking_loss_grad(W, H, color.data_ptr(), depth.data_ptr(), target_color.data_ptr(),
                              target_depth.data_ptr(), float(lam[0]), float(lam[1]), dcolor.data_ptr(),
                              ddepth.data_ptr(), _ptr(loss), _stream())
    return dcolor, ddepth


def mapping_loss_grad(color, depth, uncertainty, target_color, target_depth, loss=None):
    """Gradient images of mean|I^ - I|_1 + mean U |D^ - D| on the device."""
    H, W = depth.shape
    dcolor, ddepth, dunc = torch.empty_like(color), torch.empty_like(depth), torch.empty_like(depth)
    B.cgsr_mapping_loss_grad(W, H, color.data_ptr(), depth.data_ptr(), uncertainty.data_ptr(),
                             target_color.data_ptr(), target_depth.data_ptr(), dcolor.data_ptr(), ddepth.data_ptr(),
                             dunc.data_ptr(), _ptr(loss), _stream())
    return dict(color=dcolor, depth=ddepth, uncertainty=dunc)


def autotune_tracking(state: State, scene: dict, poses: torch.Tensor, cams, target_colors, target_depths,
                      repeats: int = 5):
    """Pick the blend kernels' pixels per lane for this tracking workload (the
    library times each candidate); the state keeps the choice.  Returns
    (fwd_pixels_per_lane, bwd_pixels_per_lane)."""
    if isinstance(cams, dict):
        cams = [cams]
    V = len(cams)
    poses = poses.reshape(V, 12)
    s = B.cgsr_autotune_tracking(state.handle, gaussians_struct(scene), V, poses.data_ptr(),
                                 [camera_struct(c) for c in cams], [t.data_ptr() for t in target_colors],
                                 [t.data_ptr() for t in target_depths], int(repeats), _stream())
    state.settings = s
    return int(s.fwd_pixels_per_lane), int(s.bwd_pixels_per_lane)


def adam_params(lr_rho=TRACK_LR_RHO, lr_phi=TRACK_LR_PHI, betas=(0.9, 0.999), eps=1e-8) -> B.cgsr_adam_params:
    return B.cgsr_adam_params(float(lr_rho), float(lr_phi), float(betas[0]), float(betas[1]), float(eps))


def pose_adam_step(poses, dposes, adam, lr_rho=TRACK_LR_RHO, lr_phi=TRACK_LR_PHI, betas=(0.9, 0.999), eps=1e-8):
    """In-place Adam step plus left retraction of every view's pose on the device."""
    V = poses.reshape(-1, 12).shape[0]
    B.cgsr_pose_adam_step(V, poses.data_ptr(), dposes.data_ptr(), adam.data_ptr(),
                          adam_params(lr_rho, lr_phi, betas, eps), _stream())


def tracking_step(state: State, scene: dict, poses: torch.Tensor, cams, target_colors, target_depths,
                  lam=TRACK_LAMBDA, dposes=None, adam=None, params=None, loss=None):
    """One fused tracking iteration of ``len(cams)`` frames (render, tracking
    loss gradient inside the blend, pose-only backward, optional Adam)."""
    if isinstance(cams, dict):
        cams = [cams]
    V = len(cams)
    poses = poses.reshape(V, 12)
    _check_f32("poses", poses)
    g = gaussians_struct(scene)
    for v, c in enumerate(cams):
        _check_f32(f"target_color[{v}]", target_colors[v], (3, int(c["height"]), int(c["width"])))
        _check_f32(f"target_depth[{v}]", target_depths[v], (int(c["height"]), int(c["width"])))
    if adam is not None and params is None:
        params = adam_params()
    B.cgsr_tracking_step(state.handle, g, V, poses.data_ptr(), [camera_struct(c) for c in cams],
                         [t.data_ptr() for t in target_colors], [t.data_ptr() for t in target_depths],
                         float(lam[0]), float(lam[1]), _ptr(dposes), _ptr(adam), params, _ptr(loss), _stream())
    state.n_views, state.n = V, g.n
    state.inputs = (scene, poses, target_colors, target_depths)


class RasterizeFunction(torch.autograd.Function):
    """Differentiable single-view render.

    Inputs: the five Gaussian parameter tensors, ``xi`` (a zero float32[6]
    tangent probe at the pose: its gradient is dL/dxi of T <- exp(xi^) T; its
    value is not read), the pose float32[12], the camera dict, the sensor
    depth (or None) and a :class:`State`.  Outputs: colour, depth, opacity,
    median depth and uncertainty (a zero-size tensor without sensor depth).
    """

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, rgb, xi, pose, cam, depth_obs, state):
        scene = dict(means=means.detach().contiguous(), log_scales=log_scales.detach().contiguous(),
                     quats=quats.detach().contiguous(), opacity_logits=opacity_logits.detach().contiguous(),
                     rgb=rgb.detach().contiguous())
        pose = pose.detach().contiguous()
        d = None if depth_obs is None else depth_obs.detach().contiguous()
        out = render(state, scene, pose, [cam], None if d is None else [d])[0]
        ctx.state = state
        ctx.keep = (scene, pose, d)
        ctx.generation = getattr(state, "generation", 0) + 1
        state.generation = ctx.generation
        unc = out.get("uncertainty")
        if unc is None:
            unc = torch.zeros(0, device=means.device)
        return out["color"], out["depth"], out["opacity"], out["depth_median"], unc

    @staticmethod
    def backward(ctx, gc, gd, go, gm, gu):
        state = ctx.state
        if getattr(state, "generation", 0) != ctx.generation:
            raise RuntimeError("the state was reused by another render before this backward; "
                               "use a separate State per outstanding forward")
        dimg = dict(color=gc, depth=gd, opacity=go, depth_median=gm,
                    uncertainty=gu if (gu is not None and gu.numel()) else None)
        need_params = any(ctx.needs_input_grad[:5])
        grads, dposes = backward(state, [dimg], param_grads=need_params, pose_grads=ctx.needs_input_grad[5])
        g = [None] * 5 if grads is None else [grads[k] for k in PARAM_NAMES]
        return (*g, None if dposes is None else dposes[0], None, None, None, None)


def rasterize(scene: dict, pose: torch.Tensor, cam: dict, depth_obs=None, xi=None, state: State | None = None):
    """Autograd entry point; returns the dict of maps of one view."""
    state = state or State()
    if xi is None:
        xi = torch.zeros(6, device=pose.device, dtype=torch.float32)
    outs = RasterizeFunction.apply(scene["means"], scene["log_scales"], scene["quats"], scene["opacity_logits"],
                                   scene["rgb"], xi, pose, cam, depth_obs, state)
    res = dict(zip(MAP_NAMES, outs))
    if depth_obs is None:
        res["uncertainty"] = None
    return res


@dataclass
class TrackingProblem:
    scene: dict
    cam: dict
    target_color: torch.Tensor
    target_depth: torch.Tensor
    lam: tuple = TRACK_LAMBDA
    lr_rho: float = TRACK_LR_RHO
    lr_phi: float = TRACK_LR_PHI


_hip_runtime = None


def upload_graph(graph: torch.cuda.CUDAGraph):
    """Uploads a captured graph's executable to the device without running
    it (hipGraphUpload on the current stream), so that its first replay starts
    as fast as later ones."""
    global _hip_runtime
    if _hip_runtime is None:
        import ctypes
        _hip_runtime = ctypes.CDLL("libamdhip64.so.7")   # the HIP runtime torch has loaded
        _hip_runtime.hipGraphUpload.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    rc = _hip_runtime.hipGraphUpload(graph.raw_cuda_graph_exec(), _stream())
    if rc != 0:
        raise RuntimeError(f"hipGraphUpload failed with error {rc}")


class TrackingSolver:
    """Sequential tracking (Eq. 20) of one frame: ``iters`` iterations of
    render -> tracking-loss gradient images -> pose-only backward -> Adam +
    retraction, captured once into a HIP graph and replayed.  The host does no
    work inside the loop."""

    def __init__(self, prob: TrackingProblem, iters: int = 50, pair_margin: float = 1.5, use_graph: bool = True,
                 reset_pose: torch.Tensor | None = None, fused: bool = True, fwd_ppl: int | None = None,
                 bwd_ppl: int | None = None, count_work: bool = False):
        """reset_pose: if given, every solve (and every graph replay) starts
        from this pose with fresh Adam moments; the reset is part of the graph.
        count_work: keep the per-pixel work counts of ``state.stats()`` (off:
        the fused step skips that bookkeeping)."""
        self.prob = prob
        self.iters = int(iters)
        cam = prob.cam
        H, W = int(cam["height"]), int(cam["width"])
        dev = prob.target_depth.device
        # pose, Adam moments and pose gradient in one buffer (16-byte aligned
        # views), so that a reset is one elementwise kernel
        self._buf = torch.zeros(12 + 16 + 6, dtype=torch.float32, device=dev)
        self.pose = self._buf[0:12]
        self.adam = self._buf[12:28].view(1, 16)
        self.dpose = self._buf[28:34].view(1, 6)
        self.dcolor = torch.empty((3, H, W), dtype=torch.float32, device=dev)
        self.ddepth = torch.empty((H, W), dtype=torch.float32, device=dev)
        self.color = torch.empty((3, H, W), dtype=torch.float32, device=dev)
        self.depth = torch.empty((H, W), dtype=torch.float32, device=dev)
        self.state = State(sync_capacity=True, fwd_ppl=fwd_ppl, bwd_ppl=bwd_ppl, count_work=count_work)
        self.g = gaussians_struct(prob.scene)
        self.cam_s = camera_struct(cam)
        self.out_s = B.cgsr_images(self.color.data_ptr(), self.depth.data_ptr(), None, None, None)
        self.grad_s = B.cgsr_images(self.dcolor.data_ptr(), self.ddepth.data_ptr(), None, None, None)
        self.pair_margin = pair_margin
        self.graph = None
        self.use_graph = use_graph
        self.pose0 = None if reset_pose is None else reset_pose.reshape(12).clone()
        self._init = None
        if self.pose0 is not None:
            self._init = torch.zeros_like(self._buf)
            self._init[0:12] = self.pose0
        self.fused = fused
        self.params = adam_params(prob.lr_rho, prob.lr_phi)
        self.cam_arr = [self.cam_s]

    def _reset_on_device(self):
        # one elementwise kernel (start pose, zero moments and gradient): a
        # captured graph then holds no memcpy or memset nodes
        torch.mul(self._init, 1.0, out=self._buf)

    def _iteration(self):
        p = self.prob
        s = _stream()
        if self.fused:
            B.cgsr_tracking_step(self.state.handle, self.g, 1, self.pose.data_ptr(), self.cam_arr,
                                 [p.target_color.data_ptr()], [p.target_depth.data_ptr()], float(p.lam[0]),
                                 float(p.lam[1]), None, self.adam.data_ptr(), self.params, None, s)
            return
        B.cgsr_render(self.state.handle, self.g, 1, self.pose.data_ptr(), [self.cam_s], None, [self.out_s], s)
        H, W = self.depth.shape
        B.cgsr_tracking_loss_grad(W, H, self.color.data_ptr(), self.depth.data_ptr(), p.target_color.data_ptr(),
                                  p.target_depth.data_ptr(), float(p.lam[0]), float(p.lam[1]),
                                  self.dcolor.data_ptr(), self.ddepth.data_ptr(), None, s)
        B.cgsr_backward(self.state.handle, [self.grad_s], None, self.dpose.data_ptr(), s)
        B.cgsr_pose_adam_step(1, self.pose.data_ptr(), self.dpose.data_ptr(), self.adam.data_ptr(), self.params, s)

    def autotune(self, pose0: torch.Tensor, repeats: int = 10):
        """Pixels per lane for this solve, timed on the solver's own state
        (no work counts, buckets reserved as prepare() reserves them) by the
        library's autotuner; the solver keeps the pick.  Call before prepare().
        Returns (fwd_pixels_per_lane, bwd_pixels_per_lane)."""
        p = self.prob
        self.reset(pose0)
        self._iteration()                       # eager, grows the tile buckets
        torch.cuda.synchronize()
        self.state.reserve(tile_pairs=int(self.state.stats().peak_pairs * self.pair_margin) + 64)
        self.reset(pose0)
        return autotune_tracking(self.state, p.scene, self.pose, [p.cam], [p.target_color], [p.target_depth],
                                 repeats=repeats)

    def reset(self, pose0: torch.Tensor):
        self.pose.copy_(pose0.reshape(12))
        self.dpose.zero_()
        self.adam.zero_()

    def prepare(self, pose0: torch.Tensor):
        """Size the tile buckets from an eager step at pose0 and capture the
        graph.  A graph that resets its own pose is then replayed once (the
        first replay of a graph executable runs about 2 % slower than the
        ones after it, even uploaded) and the pose set back to pose0; a
        bucket overflow in that replay is reported by the next check()."""
        self.reset(pose0)
        self._iteration()                       # eager, grows the tile buckets
        torch.cuda.synchronize()
        st = self.state.stats()
        self.state.reserve(tile_pairs=int(st.peak_pairs * self.pair_margin) + 64)
        self.reset(pose0)
        if self.use_graph:
            self.graph = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                with torch.cuda.graph(self.graph, stream=side):
                    if self.pose0 is not None:
                        self._reset_on_device()
                    for _ in range(self.iters):
                        self._iteration()
            torch.cuda.current_stream().wait_stream(side)
            upload_graph(self.graph)
            if self.pose0 is not None:
                self.graph.replay()
                self.reset(pose0)
            torch.cuda.synchronize()

    def run(self):
        """One solve of ``iters`` iterations from the current pose."""
        if self.graph is not None:
            self.graph.replay()
        else:
            if self.pose0 is not None:
                self._reset_on_device()
            for _ in range(self.iters):
                self._iteration()

    def check(self):
        self.state.check()
