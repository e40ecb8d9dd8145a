"""Seeded synthetic inputs shaped like the paper's indoor RGB-D workloads.

This module only draws numbers: Gaussian parameter sets, camera intrinsics,
world->camera poses and target images.  It holds none of the rasterizer's
arithmetic, so both the FP64 oracle (through the tests) and the HIP path use
it as their common, independent source of inputs.

Conventions shared with every consumer:

* Gaussian parameters are float32 SoA arrays: ``means[n,3]``, ``log_scales[n,3]``,
  ``quats[n,4]`` in (w, x, y, z) order (not necessarily unit length),
  ``opacity_logits[n]`` and ``rgb[n,3]``.  Scale is stored as its log and
  opacity as its logit (Sec. 3.1, Eq. 1 parameterised so gradient steps keep
  the covariance positive semi-definite).
* A pose is a world->camera rigid transform ``(R[3,3], t[3])`` with OpenCV
  camera axes: x right, y down, z forward.
* A camera is ``dict(width, height, fx, fy, cx, cy)``; pixel centres sit at
  integer coordinates.

The paper measures on Replica, TUM-RGBD and ScanNet (Sec. 4); none of those
sequences is reproduced here.  Rooms of points on box walls stand in for them.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "camera",
    "uniform_box_scene",
    "room_scene",
    "level_room_pose",
    "perturb_pose",
    "random_walk_poses",
    "random_targets",
    "tracking_frames",
    "TRACKING_RESOLUTIONS",
    "rot_about_axis",
    "TRACKING_CAMERA",
    "MAPPING_CAMERA",
    "SMALL_CAMERA",
]


def camera(width: int, height: int, fx: float, fy: float, cx: float, cy: float) -> dict:
    return dict(width=int(width), height=int(height), fx=float(fx), fy=float(fy),
                cx=float(cx), cy=float(cy))


#: 64x48 parity camera (f = 60, principal point (32, 24)).
SMALL_CAMERA = camera(64, 48, 60.0, 60.0, 32.0, 24.0)
#: 640x480 tracking camera (f = 525, principal point (320, 240)).
TRACKING_CAMERA = camera(640, 480, 525.0, 525.0, 320.0, 240.0)
#: 1200x680 mapping camera (f = 600, principal point (600, 340)).
MAPPING_CAMERA = camera(1200, 680, 600.0, 600.0, 600.0, 340.0)


def _random_unit_quats(rng: np.random.Generator, n: int) -> np.ndarray:
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _pack(means, log_scales, quats, opacity_logits, rgb) -> dict:
    f = np.float32
    return dict(
        means=np.ascontiguousarray(means, dtype=f),
        log_scales=np.ascontiguousarray(log_scales, dtype=f),
        quats=np.ascontiguousarray(quats, dtype=f),
        opacity_logits=np.ascontiguousarray(opacity_logits, dtype=f),
        rgb=np.ascontiguousarray(rgb, dtype=f),
    )


def uniform_box_scene(seed: int, n: int = 2000, *, xy=(-1.0, 1.0), z=(1.5, 4.0),
                      log_scale=(-3.5, 0.5), opacity=(0.0, 1.0)) -> dict:
    """Gaussians in a box in front of an identity camera.

    Draw order (fixed): x, y, z, log-scales, quaternions, opacity logits, rgb.
    Means: x, y ~ U[xy], z ~ U[z].  Log-scales ~ N(mean, std) per axis.
    Quaternions: normalise(N(0, I4)).  Opacity logit ~ N(mean, std), so the
    opacity is sigmoid of a normal draw.  RGB ~ U[0, 1].
    """
    rng = np.random.default_rng(seed)
    x = rng.uniform(xy[0], xy[1], n)
    y = rng.uniform(xy[0], xy[1], n)
    zz = rng.uniform(z[0], z[1], n)
    ls = rng.normal(log_scale[0], log_scale[1], (n, 3))
    q = _random_unit_quats(rng, n)
    o = rng.normal(opacity[0], opacity[1], n)
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    return _pack(np.stack([x, y, zz], 1), ls, q, o, rgb)


def sh_coefficients(seed: int, n: int, degree: int, *, dc=(-1.5, 1.5), rest_std: float = 0.3) -> np.ndarray:
    """View-dependent colour coefficients [n, (degree + 1)^2, 3] float32.

    Draw order (fixed): the degree-0 coefficients ~ U[dc], then the others ~
    N(0, rest_std), each in [n, K, 3] order.  Inputs only: how they turn into
    a colour is the library's business."""
    rng = np.random.default_rng(seed)
    K = (degree + 1) ** 2
    out = np.empty((n, K, 3), np.float32)
    out[:, 0, :] = rng.uniform(dc[0], dc[1], (n, 3))
    if K > 1:
        out[:, 1:, :] = rng.normal(0.0, rest_std, (n, K - 1, 3))
    return out


def room_scene(seed: int, n: int, dims=(5.0, 4.0, 3.0), *, jitter: float = 0.01,
               log_scale=(-4.0, 0.4), opacity=(1.0, 1.0)) -> dict:
    """Gaussians on the six walls of an axis-aligned room centred at the origin, z up.

    Points are split over the faces multinomially by face area and are uniform
    on each face, then jittered by N(0, jitter) per axis.  Draw order (fixed):
    face counts, per-face uniform coordinates (faces in the order -x, +x, -y,
    +y, -z, +z), jitter, log-scales, quaternions, opacity logits, rgb.
    """
    rng = np.random.default_rng(seed)
    L, W, H = (float(v) for v in dims)
    areas = np.array([W * H, W * H, L * H, L * H, L * W, L * W])
    counts = rng.multinomial(n, areas / areas.sum())
    pts = []
    half = np.array([L, W, H]) / 2.0
    for face, c in enumerate(counts):
        axis, sign = face // 2, (-1.0 if face % 2 == 0 else 1.0)
        p = rng.uniform(-1.0, 1.0, (c, 3)) * half
        p[:, axis] = sign * half[axis]
        pts.append(p)
    means = np.concatenate(pts, 0)
    means = means + rng.normal(0.0, jitter, means.shape)
    ls = rng.normal(log_scale[0], log_scale[1], (n, 3))
    q = _random_unit_quats(rng, n)
    o = rng.normal(opacity[0], opacity[1], n)
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    return _pack(means, ls, q, o, rgb)


def _pose_from_center_axes(center, right, down, forward):
    # Rows of the world->camera rotation are the camera axes in world coordinates.
    R = np.stack([right, down, forward], 0)
    t = -R @ np.asarray(center, dtype=np.float64)
    return R, t


def level_room_pose(seed: int, radius: float = 1.0):
    """A level camera inside the room: position uniform in the ball of
    ``radius`` about the centre, yaw ~ U[0, 2pi), no pitch or roll.

    Returns ``(R, t)`` world->camera in float64.
    """
    rng = np.random.default_rng(seed)
    while True:  # rejection sampling of a point in the ball
        c = rng.uniform(-radius, radius, 3)
        if c @ c <= radius * radius:
            break
    yaw = rng.uniform(0.0, 2.0 * np.pi)
    fwd = np.array([np.cos(yaw), np.sin(yaw), 0.0])
    right = np.array([np.sin(yaw), -np.cos(yaw), 0.0])
    down = np.array([0.0, 0.0, -1.0])
    return _pose_from_center_axes(c, right, down, fwd)


def rot_about_axis(axis, angle: float) -> np.ndarray:
    """Rotation matrix by ``angle`` radians about unit ``axis`` (input recipe helper)."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return np.eye(3) + np.sin(angle) * K + (1.0 - np.cos(angle)) * (K @ K)


def perturb_pose(R, t, seed: int, trans_std: float = 0.02, rot_deg: float = 1.0):
    """Start pose for a tracking solve: the camera centre moves by N(0, trans_std)
    per axis and the camera turns by ``rot_deg`` about a random axis."""
    rng = np.random.default_rng(seed)
    dc = rng.normal(0.0, trans_std, 3)
    axis = rng.standard_normal(3)
    dR = rot_about_axis(axis, np.deg2rad(rot_deg))
    R = np.asarray(R, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    center = -R.T @ t + dc
    R2 = dR @ R
    return R2, -R2 @ center


def random_walk_poses(seed: int, n_views: int, dims=(8.0, 6.0, 3.0), step: float = 0.3,
                      turn_deg: float = 15.0, wall_margin: float = 0.5):
    """Keyframe poses along a seeded random walk from the room centre: each step
    moves the camera ``step`` metres in a random direction (reflected to stay
    ``wall_margin`` inside the walls) and turns it ``turn_deg`` about a random axis.
    The first pose is level with a random yaw."""
    rng = np.random.default_rng(seed)
    R0, t0 = level_room_pose(int(rng.integers(1 << 30)), radius=0.0)
    R = R0
    c = np.zeros(3)
    lim = np.array(dims, dtype=np.float64) / 2.0 - wall_margin
    out = [(R.copy(), -R @ c)]
    for _ in range(n_views - 1):
        d = rng.standard_normal(3)
        c = c + step * d / np.linalg.norm(d)
        for k in range(3):  # reflect at the margin box
            if c[k] > lim[k]:
                c[k] = 2 * lim[k] - c[k]
            if c[k] < -lim[k]:
                c[k] = -2 * lim[k] - c[k]
        R = rot_about_axis(rng.standard_normal(3), np.deg2rad(turn_deg)) @ R
        out.append((R.copy(), -R @ c))
    return out


def random_targets(seed: int, cam: dict, depth_range=(1.5, 4.0)):
    """Random target colour [3,H,W] ~ U[0,1] and depth [H,W] ~ U[depth_range] (float32)."""
    rng = np.random.default_rng(seed)
    H, W = cam["height"], cam["width"]
    color = rng.uniform(0.0, 1.0, (3, H, W)).astype(np.float32)
    depth = rng.uniform(depth_range[0], depth_range[1], (H, W)).astype(np.float32)
    return color, depth


#: Frame sizes of the many-frame tracking workload.
TRACKING_RESOLUTIONS = ((320, 240), (640, 480), (960, 540), (1200, 680))


def tracking_frames(seed: int, n_frames: int, radius: float = 1.0):
    """Independent tracking frames of uneven resolution: each frame draws its
    size uniformly from TRACKING_RESOLUTIONS, its focal length scales with the
    width (f = 525 W / 640), its principal point is the image centre, and its
    pose is a level room pose (level_room_pose) of its own seed.
    Returns a list of (camera, (R, t))."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_frames):
        W, H = TRACKING_RESOLUTIONS[int(rng.integers(len(TRACKING_RESOLUTIONS)))]
        f = 525.0 * W / 640.0
        cam = camera(W, H, f, f, W / 2.0, H / 2.0)
        out.append((cam, level_room_pose(int(rng.integers(1 << 30)), radius)))
    return out
