"""FP64 oracle of Gaussian management (Sec. 3.3) -- TEST INFRASTRUCTURE.

Written from the definitions in plain numpy, each function in the order of
the method's steps:

* spawning: pixels whose rendered opacity (Eq. 9) is below psi = 0.5 are
  unobserved or under-reconstructed; each with a sensor depth becomes a new
  Gaussian from its colour and depth (with no opacity map every pixel with a
  depth spawns: the dense first-frame initialisation);
* removal: the set is compacted to the Gaussians kept, in order;
* densification, kept from the splatting method the paper builds on: a
  Gaussian whose mean screen-space gradient reaches a threshold is cloned
  when small and split in two when large.

Readings where the paper is silent (also stated in the library's header):
* a spawned Gaussian sits at the back-projection of the pixel centre at its
  sensor depth, is isotropic with scale D / ((fx + fy) / 2) (one pixel's
  footprint at that depth), has the identity rotation, the caller's opacity
  logit and the pixel's colour (with view-dependent colour: the degree-0
  coefficient (c - 1/2) / Y_00, the others zero); pixels are taken in
  row-major order, optionally on a grid of stride s (u and v multiples of s);
* the densification statistic of a Gaussian is the sum over renders and
  views in which it reaches the image of |dL/dmu| (its projected mean, in
  pixels), divided by the number of those; with no such render it is zero;
  a Gaussian is "small" if its largest scale is at most dense_scale;
* a split replaces Gaussian i by two at mu_i + R_i diag(s_i) z_ik (z_ik the
  caller's standard normal draws, k = 0, 1) with scales s_i / 1.6 and the
  other parameters copied; the new set is the Gaussians that were not split,
  in order, then the clones in index order, then the split halves in index
  order (k = 0 before k = 1).
"""
from __future__ import annotations

import numpy as np

#: Opacity threshold below which a rendered pixel counts as unobserved (Sec. 3.3).
SPAWN_PSI = 0.5
#: Scale divisor of a split (two children, each 1 / (0.8 * 2) of the parent).
SPLIT_SCALE_DIV = 1.6


def quat_to_rot(q):
    """Rotation of the normalised quaternion (w, x, y, z)."""
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def spawn(color, depth, cam, pose, opacity=None, psi=SPAWN_PSI, init_logit=0.0, stride=1, sh_degree=None):
    """New Gaussians from the pixels of one RGB-D view (see the module
    readings).  color [3, H, W], depth [H, W], opacity [H, W] or None; pose
    (R, t) world -> camera.  Returns a dict of parameter arrays (rgb, or sh
    [m, K, 3] when sh_degree is given) and the spawning pixels' flat indices."""
    H, W = depth.shape
    R, t = (np.asarray(a, np.float64) for a in pose)
    fx, fy, cx, cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    means, scales, cols, idx = [], [], [], []
    for v in range(0, H, stride):
        for u in range(0, W, stride):
            D = float(depth[v, u])
            if not D > 0.0:
                continue
            if opacity is not None and not float(opacity[v, u]) < psi:
                continue
            p_cam = D * np.array([(u - cx) / fx, (v - cy) / fy, 1.0])
            means.append(R.T @ (p_cam - t))
            scales.append(D / (0.5 * (fx + fy)))
            cols.append(np.asarray(color[:, v, u], np.float64))
            idx.append(v * W + u)
    m = len(idx)
    out = dict(means=np.array(means).reshape(m, 3),
               log_scales=np.repeat(np.log(np.array(scales)).reshape(m, 1), 3, 1),
               quats=np.tile([1.0, 0.0, 0.0, 0.0], (m, 1)),
               opacity_logits=np.full(m, float(init_logit)))
    cols = np.array(cols).reshape(m, 3)
    if sh_degree is None:
        out["rgb"] = cols
    else:
        sh = np.zeros((m, (sh_degree + 1) ** 2, 3))
        sh[:, 0, :] = (cols - 0.5) * np.sqrt(4.0 * np.pi)     # Y_00 = 1 / sqrt(4 pi)
        out["sh"] = sh
    return out, np.array(idx, np.int64)


def compact(params: dict, keep):
    """The Gaussians with keep != 0, in order."""
    k = np.asarray(keep).astype(bool)
    return {name: a[k] for name, a in params.items()}


def densify_statistic(grad_accum, denom):
    """Mean screen-space gradient norm per Gaussian (0 without renders)."""
    d = np.asarray(denom, np.float64)
    return np.where(d > 0, np.asarray(grad_accum, np.float64) / np.maximum(d, 1), 0.0)


def densify(params: dict, grad_accum, denom, grad_threshold, dense_scale, normals):
    """Clone small and split large Gaussians whose statistic reaches the
    threshold.  normals: [n, 2, 3] standard normal draws (only those of split
    Gaussians are used).  Returns (new parameter dict, clone mask, split mask)."""
    stat = densify_statistic(grad_accum, denom)
    smax = np.exp(np.asarray(params["log_scales"], np.float64)).max(1)
    hot = stat >= grad_threshold
    clone = hot & (smax <= dense_scale)
    split = hot & (smax > dense_scale)
    kept = compact(params, ~split)
    clones = compact(params, clone)
    ids = np.nonzero(split)[0]
    halves = {k: [] for k in params}
    for i in ids:
        Ri = quat_to_rot(params["quats"][i])
        s = np.exp(np.asarray(params["log_scales"][i], np.float64))
        for k in range(2):
            for name in params:
                if name == "means":
                    halves[name].append(np.asarray(params["means"][i], np.float64) + Ri @ (s * normals[i, k]))
                elif name == "log_scales":
                    halves[name].append(np.asarray(params["log_scales"][i], np.float64) - np.log(SPLIT_SCALE_DIV))
                else:
                    halves[name].append(np.asarray(params[name][i], np.float64))
    out = {}
    for name in params:
        parts = [np.asarray(kept[name], np.float64), np.asarray(clones[name], np.float64)]
        if len(ids):
            parts.append(np.array(halves[name]))
        out[name] = np.concatenate([p.reshape((-1,) + np.asarray(params[name]).shape[1:]) for p in parts], 0)
    return out, clone, split
