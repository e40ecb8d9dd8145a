"""FP64 oracle of the mapping objective, Eq. 18 -- TEST INFRASTRUCTURE.

Each term is written from its definition (Sec. 3.2-3.3) on whole images in
float64: the colour L1 (Eq. 14), structural similarity (Eq. 15), depth L1
(Eq. 16), depth alignment (Eq. 12), scale isotropy (Eq. 17) and geometry
variance (Eq. 11).  Gradients of the image terms are the subgradients written
out; the SSIM gradient is PyTorch autograd of the plain float64 definition on
the CPU.

Readings where the paper is silent:
* SSIM uses the 3D Gaussian splatting conventions it inherits: an 11x11
  Gaussian window of standard deviation 1.5 (normalised), zero padding,
  C1 = 0.01^2, C2 = 0.03^2, the mean over channels and pixels; the loss term
  is 1 - SSIM (the similarity itself is to be maximised).
* Eq. 12 runs over pixels that have a median Gaussian (Eq. 8); a pixel
  whose transmittance never falls below 0.5 has no median depth and adds
  nothing, while the mean still divides by H W.
* Eq. 17 averages over the Gaussians visible in the view (those that reach
  the image); with epsilon = 1 the ratio of largest to smallest scale is
  never below epsilon, and ties pick the first axis.
* The window's objective is the sum over its keyframes of Eq. 18.
"""
from __future__ import annotations

import numpy as np

#: Eq. 18 weights for Replica (Sec. 4): colour, ssim, geo, align, iso, var.
OMEGA_REPLICA = (0.7, 0.1, 0.25, 0.25, 0.1, 0.15)
#: Eq. 18 weights for TUM and ScanNet (Sec. 4).
OMEGA_REAL = (1.0, 0.1, 0.8, 0.5, 0.1, 0.5)
#: Eq. 17 anisotropy level (Sec. 3.3).
ISO_EPS = 1.0
SSIM_WINDOW = 11
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def gaussian_window_1d(size=SSIM_WINDOW, sigma=SSIM_SIGMA):
    x = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-x * x / (2.0 * sigma * sigma))
    return g / g.sum()


def _ssim_torch(x, y):
    """Mean SSIM of two [C, H, W] float64 torch tensors (Eq. 15)."""
    import torch
    import torch.nn.functional as F
    C = x.shape[0]
    g = torch.from_numpy(gaussian_window_1d())
    w2 = torch.outer(g, g).expand(C, 1, SSIM_WINDOW, SSIM_WINDOW).contiguous()
    pad = SSIM_WINDOW // 2

    def blur(z):
        return F.conv2d(z.unsqueeze(0), w2, padding=pad, groups=C)[0]
    mx, my = blur(x), blur(y)
    sxx = blur(x * x) - mx * mx
    syy = blur(y * y) - my * my
    sxy = blur(x * y) - mx * my
    s = ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)) / ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2))
    return s.mean(), s


def ssim(x, y):
    """Mean SSIM and the per-pixel SSIM map of [C, H, W] images."""
    import torch
    m, s = _ssim_torch(torch.from_numpy(np.asarray(x, np.float64)), torch.from_numpy(np.asarray(y, np.float64)))
    return float(m), s.numpy()


def ssim_loss(x, y):
    """L_ssim = 1 - SSIM(x, y) and its gradient with respect to x."""
    import torch
    xt = torch.from_numpy(np.array(x, np.float64)).requires_grad_(True)
    m, _ = _ssim_torch(xt, torch.from_numpy(np.asarray(y, np.float64)))
    loss = 1.0 - m
    loss.backward()
    return float(loss.detach()), xt.grad.numpy()


def color_l1(color, target):
    """Eq. 14: L1 over channels, mean over pixels."""
    hw = color.shape[-1] * color.shape[-2]
    d = np.asarray(color, np.float64) - np.asarray(target, np.float64)
    return np.abs(d).sum() / hw, np.sign(d) / hw


def geo_l1(depth, target):
    """Eq. 16."""
    hw = depth.shape[-1] * depth.shape[-2]
    d = np.asarray(depth, np.float64) - np.asarray(target, np.float64)
    return np.abs(d).sum() / hw, np.sign(d) / hw


def align_loss(depth, depth_median, has_median):
    """Eq. 12 over pixels with a median; returns (L, dL/ddepth, dL/dmedian)."""
    hw = depth.shape[-1] * depth.shape[-2]
    d = (np.asarray(depth, np.float64) - np.asarray(depth_median, np.float64)) * has_median
    g = np.sign(d) / hw
    return np.abs(d).sum() / hw, g, -g


def var_loss(uncertainty):
    """Eq. 11: mean |U|."""
    U = np.asarray(uncertainty, np.float64)
    hw = U.shape[-1] * U.shape[-2]
    return np.abs(U).sum() / hw, np.sign(U) / hw


def iso_loss(log_scales, visible, eps=ISO_EPS):
    """Eq. 17 over the visible Gaussians; returns (L, dL/dlog_scales [n, 3])."""
    ls = np.asarray(log_scales, np.float64)
    vis = np.asarray(visible).astype(bool)
    g = np.zeros_like(ls)
    nvis = int(vis.sum())
    if nvis == 0:
        return 0.0, g
    imax = np.argmax(ls, axis=1)
    imin = np.argmin(ls, axis=1)
    rows = np.arange(ls.shape[0])
    r = np.exp(ls[rows, imax] - ls[rows, imin])     # max s / min s
    term = np.maximum(r, eps) - eps
    active = vis & (r > eps)
    np.add.at(g, (rows[active], imax[active]), r[active] / nvis)
    np.add.at(g, (rows[active], imin[active]), -r[active] / nvis)
    return term[vis].sum() / nvis, g


def mapping_objective(maps, target_color, target_depth, log_scales, visible, omega=OMEGA_REPLICA):
    """Eq. 18 for one keyframe.  maps: color, depth, depth_median, uncertainty
    and has_median (bool [H, W]).  Returns (L, dimg dict, dlog_scales)."""
    w1, w2, w3, w4, w5, w6 = omega
    lc, gc = color_l1(maps["color"], target_color)
    ls, gs = ssim_loss(maps["color"], target_color)
    lg, gg = geo_l1(maps["depth"], target_depth)
    la, gad, gam = align_loss(maps["depth"], maps["depth_median"], maps["has_median"])
    li, gi = iso_loss(log_scales, visible)
    lv, gv = var_loss(maps["uncertainty"])
    L = w1 * lc + w2 * ls + w3 * lg + w4 * la + w5 * li + w6 * lv
    dimg = dict(color=w1 * gc + w2 * gs, depth=w3 * gg + w4 * gad, depth_median=w4 * gam, uncertainty=w6 * gv)
    return L, dimg, w5 * gi
