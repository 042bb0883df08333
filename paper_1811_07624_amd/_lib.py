"""ctypes marshalling for libhh.so (declared in include/hh.h).

Only argument marshalling lives here: tensors are passed as device pointers
with their leading dimensions, on torch's current stream.  Every computation
happens in the HIP library; if it is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhh.so")

HH_OK, HH_ERR_INVALID_ARG, HH_ERR_UNSUPPORTED, HH_ERR_WORKSPACE, HH_ERR_HIP = range(5)
HH_F64, HH_F32, HH_BF16, HH_F16 = range(4)
HH_ALGO_AUTO, HH_ALGO_FUSED, HH_ALGO_WY, HH_ALGO_FUSED_QR = range(4)
(HH_OP_APPLY, HH_OP_APPLY_T, HH_OP_SYM, HH_OP_MAHAL, HH_OP_APPLY_BWD, HH_OP_APPLY_T_BWD,
 HH_OP_SYM_BWD, HH_OP_MAHAL_BWD) = range(8)

EXPORTS = (
    "hh_workspace_size", "hh_apply", "hh_apply_T", "hh_sym_apply", "hh_mahalanobis",
    "hh_apply_backward", "hh_apply_T_backward", "hh_sym_apply_backward",
    "hh_mahalanobis_backward", "hh_saved_size", "hh_forward_save", "hh_backward_saved",
    "hh_forward_signed", "hh_backward_signed", "hh_forward_noalloc", "hh_factor_workspace_size",
    "hh_factor_orthonormal", "hh_shf_workspace_size", "hh_shf", "hh_knn_workspace_size", "hh_knn",
    "hh_mahalanobis_saved_size", "hh_mahalanobis_save", "hh_mahalanobis_backward_saved",
    "hh_status_string",
    "hh_last_error", "hh_version",
)
HH_FACTOR_CONSTRAINED, HH_FACTOR_UNCONSTRAINED, HH_FACTOR_QR = range(3)

# Bytes of the library's static scratch used by hh_forward_noalloc.
NOALLOC_SCRATCH_BYTES = 16 << 20

_TORCH_TO_HH = {torch.float64: HH_F64, torch.float32: HH_F32, torch.bfloat16: HH_BF16,
                torch.float16: HH_F16}
_ALGOS = {"auto": HH_ALGO_AUTO, "fused": HH_ALGO_FUSED, "wy": HH_ALGO_WY,
          "fused_qr": HH_ALGO_FUSED_QR}


class HHDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("h", ctypes.c_int64), ("N", ctypes.c_int64),
                ("param_dtype", ctypes.c_int), ("io_dtype", ctypes.c_int),
                ("compute_dtype", ctypes.c_int), ("algo", ctypes.c_int)]


class HHError(RuntimeError):
    def __init__(self, fn, status, detail):
        self.status = status
        super().__init__(f"{fn} failed: {detail}")


_lib = None


def lib():
    """Load libhh.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with python -m paper_1811_07624_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, I, S = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
    D = ctypes.POINTER(HHDesc)
    sig = {
        "hh_workspace_size": [ctypes.c_int, D, ctypes.POINTER(S)],
        "hh_apply": [D, P, I, P, I, P, I, P, S, P],
        "hh_apply_T": [D, P, I, P, I, P, I, P, S, P],
        "hh_sym_apply": [D, P, I, P, P, I, P, I, P, S, P],
        "hh_mahalanobis": [D, P, I, P, P, I, P, I, P, P, S, P],
        "hh_apply_backward": [D, P, I, P, I, P, I, P, I, P, I, P, S, P],
        "hh_apply_T_backward": [D, P, I, P, I, P, I, P, I, P, I, P, S, P],
        "hh_sym_apply_backward": [D, P, I, P, P, I, P, I, P, I, P, I, P, P, S, P],
        "hh_mahalanobis_backward": [D, P, I, P, P, I, P, I, P, P, P, I, P, I, P, P, S, P],
        "hh_saved_size": [ctypes.c_int, D, ctypes.POINTER(S)],
        "hh_forward_save": [ctypes.c_int, D, P, I, P, P, I, P, I, P, S, P, S, P],
        "hh_backward_saved": [ctypes.c_int, D, P, I, P, P, I, P, S, P, I, P, I, P, I, P, P, S, P],
        "hh_forward_signed": [ctypes.c_int, D, P, I, P, P, P, P, I, P, I, P, I, P, S, P],
        "hh_backward_signed": [ctypes.c_int, D, P, I, P, P, P, P, I, P, I, P, I, P, P, I, P, I, P, P,
                               S, P],
        "hh_forward_noalloc": [ctypes.c_int, D, P, I, P, P, I, P, I, P, I, P],
        "hh_factor_workspace_size": [ctypes.c_int, I, I, ctypes.POINTER(S)],
        "hh_factor_orthonormal": [ctypes.c_int, I, I, P, I, P, I, P, P, P, S, P],
        "hh_shf_workspace_size": [I, I, I, ctypes.POINTER(S)],
        "hh_shf": [I, I, I, ctypes.c_int, P, I, P, I, P, P, P, P, S, P],
        "hh_knn_workspace_size": [I, I, I, I, ctypes.POINTER(S)],
        "hh_knn": [I, I, I, I, P, I, P, I, P, P, P, S, P],
        "hh_mahalanobis_saved_size": [D, ctypes.POINTER(S)],
        "hh_mahalanobis_save": [D, P, I, P, P, I, P, I, P, P, S, P, S, P],
        "hh_mahalanobis_backward_saved": [D, P, I, P, P, I, P, I, P, S, P, P, P, I, P, I, P, P, S, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.hh_status_string.argtypes = [ctypes.c_int]
    L.hh_status_string.restype = ctypes.c_char_p
    L.hh_last_error.argtypes = []
    L.hh_last_error.restype = ctypes.c_char_p
    L.hh_version.restype = ctypes.c_int
    _lib = L
    return L


def check(fn: str, status: int) -> None:
    if status != HH_OK:
        L = lib()
        raise HHError(fn, status, "%s: %s" % (L.hh_status_string(status).decode(),
                                              L.hh_last_error().decode()))


def hh_dtype(t: torch.dtype) -> int:
    try:
        return _TORCH_TO_HH[t]
    except KeyError:
        raise TypeError(f"unsupported dtype {t}") from None


def make_desc(n, h, N, param, io, compute, algo="auto") -> HHDesc:
    return HHDesc(int(n), int(h), int(N), hh_dtype(param), hh_dtype(io), hh_dtype(compute),
                  _ALGOS[algo])


def ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def ld(t: torch.Tensor) -> int:
    """Leading dimension of an (rows, n) tensor whose rows are contiguous (an
    empty tensor's strides mean nothing: its leading dimension is n)."""
    if t.dim() == 2 and t.numel() == 0:
        return max(int(t.shape[1]), 1)
    if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1):
        raise ValueError("expected a 2-D tensor with unit stride along its last dimension")
    return max(int(t.stride(0)), int(t.shape[1]))


def stream_of(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def saved_record(op: int, desc: HHDesc, device) -> torch.Tensor:
    """Caller-owned buffer for the coefficient record of forward op `op` (WY only)."""
    nbytes = ctypes.c_size_t(0)
    check("hh_saved_size", lib().hh_saved_size(op, ctypes.byref(desc), ctypes.byref(nbytes)))
    return torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)


# Small workspaces are kept per (device, stream) and reused: calls on one
# stream run in order, so a later call cannot overwrite scratch space an
# earlier call still uses.  Larger ones are allocated per call.
_WS_CACHE_MAX = 16 << 20
_ws_cache = {}


def workspace(op: int, desc: HHDesc, device) -> torch.Tensor:
    nbytes = ctypes.c_size_t(0)
    check("hh_workspace_size", lib().hh_workspace_size(op, ctypes.byref(desc), ctypes.byref(nbytes)))
    need = max(int(nbytes.value), 256)
    if need > _WS_CACHE_MAX:
        return torch.empty(need, dtype=torch.uint8, device=device)
    dev = torch.device(device)
    key = (dev.index if dev.index is not None else torch.cuda.current_device(),
           torch.cuda.current_stream(dev).cuda_stream)
    ws = _ws_cache.get(key)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1 << 20), dtype=torch.uint8, device=dev)
        _ws_cache[key] = ws
    return ws
