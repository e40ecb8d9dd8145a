"""Shared helpers of the test-suite (host side only)."""
import sys

import numpy as np

# Relative distance to a decision threshold under which float32 and float64
# may legitimately decide differently (alpha skip/cap, stop, median): the
# float32 alpha and transmittance carry relative errors of order 1e-6 (a
# rounded exponent of magnitude <= 8, a product of at most a few hundred
# factors), so 1e-4 leaves a factor of about 100 ...
DECISION_MARGIN = 1e-4
# ... and relative depth gap under which two Gaussians may come in either
# order.  The tiles order by the float32 depth (then the Gaussian's index, as
# the oracle breaks exact ties); rounding is monotone, so two depths keep
# their float64 order unless both round to the same float32, which needs
# |d1 - d2| < ulp(d) <= 2^-23 d.  1.2e-7 is 2^-23 (1.19e-7) rounded up.
ORDER_MARGIN = 1.2e-7

MAPS = ("color", "depth", "opacity", "depth_median", "uncertainty")


def unambiguous(ref):
    """Pixels of an oracle render whose every discrete decision is clear."""
    return ((ref["decision_margin"] >= DECISION_MARGIN) & (ref["order_margin"] >= ORDER_MARGIN)
            & (ref["stop_order_margin"] >= ORDER_MARGIN))


def order_only_ambiguous(ref):
    """Pixels whose thresholds are clear but whose blend order may swap two
    near-equal depths.  Accumulated opacity, 1 - prod(1 - alpha), does not
    depend on that order, so it must still match there."""
    return ((ref["decision_margin"] >= DECISION_MARGIN) & (ref["order_margin"] < ORDER_MARGIN)
            & (ref["stop_order_margin"] >= ORDER_MARGIN))


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _pixel_values(maps, px, n_img):
    """[n, 7] values (colour r, g, b, depth, opacity, median depth,
    uncertainty) of the flat pixels px from full maps ([3,H,W] / [H,W]) or
    from maps already flat over px ([3,n] / [n]); NaN where a map is absent."""
    px = np.asarray(px).reshape(-1)
    out = np.full((px.size, 7), np.nan)
    for k, cols in (("color", (0, 1, 2)), ("depth", (3,)), ("opacity", (4,)), ("depth_median", (5,)),
                    ("uncertainty", (6,))):
        v = maps.get(k)
        if v is None:
            continue
        v = np.asarray(v, np.float64)
        flat = v.reshape(len(cols), -1)
        out[:, list(cols)] = (flat[:, px] if flat.shape[1] == n_img and flat.shape[1] != px.size
                              else flat).T
    return out


def check_maps(gpu, scene, cam, pose, dobs=None, px=None, ref=None, tol=1e-4, max_ambiguous=None,
               label="", maps=MAPS):
    """Element-wise parity of GPU maps against the FP64 oracle on the flat
    pixels px (all pixels when None).

    gpu: maps as full images or flat over px.  Pixels whose every discrete
    decision clears DECISION_MARGIN and ORDER_MARGIN must match the oracle's
    render within tol on every map.  Every other pixel must match, within
    tol on every map at once, one of the results the oracle gives when each
    of its near-threshold decisions may go either way
    (oracle.render_alternatives: alpha skip or cap and blending stop of
    Eq. 3-5, median of Eq. 7-8, order of near-tied depths).  No pixel is
    left unchecked.  max_ambiguous bounds the fraction of pixels with
    alternatives.  Returns a dict of counts and worst errors."""
    import oracle
    H, W = int(cam["height"]), int(cam["width"])
    px = np.arange(H * W) if px is None else np.asarray(px, np.int64).reshape(-1)
    if ref is None:
        ref = oracle.render(scene, cam, pose, dobs, pixels=px)
    keep = [k for k in maps if k in gpu and gpu[k] is not None and ref.get(k) is not None]
    cols = sorted({c for k in keep for c in {"color": (0, 1, 2), "depth": (3,), "opacity": (4,),
                                              "depth_median": (5,), "uncertainty": (6,)}[k]})
    g = _pixel_values({k: gpu[k] for k in keep}, px, H * W)[:, cols]
    r = _pixel_values({k: ref[k] for k in keep}, px, H * W)[:, cols]
    clear = unambiguous(ref).reshape(-1)
    worst = np.abs(g - r)[clear].max(0) if clear.any() else np.zeros(len(cols))
    bad = clear & (np.abs(g - r).max(1) > tol)
    assert not bad.any(), (label, "clear pixels off the oracle", px[bad][:10], worst)
    amb = np.nonzero(~clear)[0]
    frac = amb.size / max(px.size, 1)
    res = dict(pixels=int(px.size), ambiguous=int(amb.size), ambiguous_frac=frac, worst_clear=worst.max(initial=0.0),
               worst_alt=0.0, over_limit=0, alternatives=0)
    if amb.size:
        alts, count = oracle.render_alternatives(scene, cam, pose, dobs, px[amb], DECISION_MARGIN, ORDER_MARGIN)
        a = alts[:, :, cols]
        n_alt = np.minimum(count, alts.shape[1])
        err = np.abs(a - g[amb][:, None, :]).max(2)                      # [n_amb, max_alts]
        err[np.arange(alts.shape[1])[None, :] >= n_alt[:, None]] = np.inf
        best = err.min(1)
        res.update(worst_alt=float(best.max()), over_limit=int((count > alts.shape[1]).sum()),
                   alternatives=int(n_alt.sum()))
        miss = best > tol
        assert not miss.any(), (label, "ambiguous pixels matching no admissible result", px[amb][miss][:10],
                                best[miss][:10], count[miss][:10])
    _say(label, "pixels", res["pixels"], "ambiguous", res["ambiguous"], f"({100 * frac:.3f} %)",
         "alternatives", res["alternatives"], "over limit", res["over_limit"],
         "worst clear err", res["worst_clear"], "worst matched-alternative err", res["worst_alt"])
    if max_ambiguous is not None:
        assert frac <= max_ambiguous, (label, frac)
    return res


def rel_l2(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def grad_parity(name, g, ref, rel=1e-3, label=""):
    """Gradient parity of one tensor: the binding bar, relative L2 error
    <= rel, asserted; and the element-wise report, the fraction of elements
    with |g - g_ref| > 1e-3 |g_ref| + 1e-5 max|g_ref| and the largest ratio
    of |g - g_ref| to that bound, printed and returned."""
    g = np.asarray(g, np.float64).ravel()
    r = np.asarray(ref, np.float64).ravel()
    e = rel_l2(g, r)
    bound = 1e-3 * np.abs(r) + 1e-5 * (np.abs(r).max() if r.size else 0.0)
    d = np.abs(g - r)
    over = d > bound
    ratio = float((d / np.where(bound > 0, bound, np.inf)).max(initial=0.0))
    frac = float(over.mean()) if r.size else 0.0
    _say(label, name, f"rel L2 {e:.3e}", f"element-wise: {100 * frac:.4f} % over 1e-3|g|+1e-5|g|_inf",
         f"(worst ratio {ratio:.2f})")
    assert e <= rel, (label, name, e)
    return frac


def identity_pose():
    return np.eye(3), np.zeros(3)


def pose12(R, t):
    return np.concatenate([np.asarray(R, np.float64).reshape(9), np.asarray(t, np.float64).reshape(3)])


_hip = None


def copy_device(dst, src_ptr: int, nbytes: int) -> None:
    """Device-to-device copy from a raw pointer the library returned into a
    torch tensor (hipMemcpy through the HIP runtime; synchronous)."""
    global _hip
    import ctypes

    import torch  # noqa: F401  (binds the soname below to torch's HIP runtime)
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so.7")  # the runtime torch already loaded
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    if nbytes <= 0:
        return
    rc = _hip.hipMemcpy(dst.data_ptr(), src_ptr, nbytes, 3)  # hipMemcpyDeviceToDevice
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed with {rc}")
