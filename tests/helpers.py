"""Shared helpers of the test-suite (host side only)."""
import numpy as np

# Relative distance to a decision threshold under which float32 and float64
# may legitimately decide differently (alpha skip/cap, stop, median) ...
DECISION_MARGIN = 1e-4
# ... and relative depth gap under which two blended Gaussians may swap order
# (the float32 camera depth carries about 2e-7 relative rounding).
ORDER_MARGIN = 1e-6


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


def rel_l2(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


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
