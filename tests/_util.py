"""Shared helpers for the test suite (error measures and device checks)."""
import numpy as np


def rel_rows(Y, Yref):
    """max_j ||y_j - yref_j|| / ||yref_j|| over rows (vectors); 0 for empty input."""
    Y = np.asarray(Y, dtype=np.float64)
    Yref = np.asarray(Yref, dtype=np.float64)
    if Y.size == 0:
        return 0.0
    num = np.linalg.norm(Y - Yref, axis=-1)
    den = np.maximum(np.linalg.norm(Yref, axis=-1), 1e-300)
    return float(np.max(num / den))


def rel_fro(A, Aref):
    A = np.asarray(A, dtype=np.float64)
    Aref = np.asarray(Aref, dtype=np.float64)
    den = max(np.linalg.norm(Aref), 1e-300)
    return float(np.linalg.norm(A - Aref) / den)


def rel_elem(d, dref):
    d = np.asarray(d, dtype=np.float64)
    dref = np.asarray(dref, dtype=np.float64)
    if d.size == 0:
        return 0.0
    return float(np.max(np.abs(d - dref) / np.maximum(np.abs(dref), 1e-300)))


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def rel_refl(dU, ref):
    """Per-reflector relative error of a gradient laid out (h, n): the max
    over reflectors k of ||dU_k - ref_k|| / max(||ref_k||, rms_k ||ref_k||).
    Measured against the reflector's own gradient, floored at the rms
    reflector-gradient norm: rounding errors of the shared products scale
    with the typical gradient, so a reflector whose gradient is unusually
    small (or exactly zero, a zero column) is not held to a tighter absolute
    bound than the others, while a wrong gradient for one reflector (an error
    of the size of its gradient) still fails, as it might not in a
    whole-tensor norm."""
    A = np.asarray(dU, dtype=np.float64)
    R = np.asarray(ref, dtype=np.float64)
    if A.size == 0:
        return 0.0
    num = np.linalg.norm(A - R, axis=-1)
    den = np.linalg.norm(R, axis=-1)
    rms = float(np.linalg.norm(R)) / np.sqrt(max(R.shape[0], 1))
    return float(np.max(num / np.maximum(np.maximum(den, rms), 1e-300)))
