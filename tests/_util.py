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
