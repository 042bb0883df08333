"""Python entry points: one torch.autograd.Function per operation of libhh.so.

Tensors use the torch view of the library's column-major layout:
  U   : (h, n)  row k is the reflector vector u_k (normalised in the library)
  X   : (N, n)  row j is vector j
  lam : (n,)
Each call passes device pointers and torch's current stream to the C ABI and
returns; no arithmetic on the data happens in Python.

``compute`` selects the arithmetic: float64/float32 run the fused
sequential-reflector kernels (data in that dtype); bfloat16/float16 run the
compact-WY matrix-core kernels (data in that dtype or in float32, which the
library rounds to the compute type and widens back; parameters in float32).
``algo`` may force "fused" or "wy"; the default "auto" follows ``compute``;
"fused_qr" runs the fused forward kernels that skip each reflector's leading
zeros (reflectors of a Householder QR, the remark after Result 3).

On the WY path a forward whose reflectors (or spectrum) need a gradient keeps
a record of its per-vector WY coefficients (h scalars per vector, not h copies
of the vector) and of its reflector setup; its backward uses them instead of a
second pass over X and a second setup.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L

_FUSED = (torch.float64, torch.float32)


def _cfg(X: torch.Tensor, compute):
    io = X.dtype
    comp = io if compute is None else compute
    param = comp if comp in _FUSED else torch.float32
    return param, io, comp


def _rows(t: torch.Tensor) -> torch.Tensor:
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if t.shape[1] > 1 and t.stride(1) != 1:
        t = t.contiguous()
    return t


def _param(t, dtype):
    if t is None:
        return None
    t = t.to(dtype)
    return t.contiguous()


def _check_dev(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("libhh operates on device tensors")


# --------------------------------------------------------------------------
# raw calls (no autograd)
# --------------------------------------------------------------------------
def is_wy(X, compute=None, algo="auto"):
    """True when a call with these arguments runs the compact-WY kernels."""
    comp = X.dtype if compute is None else compute
    return algo == "wy" or (algo == "auto" and comp not in _FUSED)


def apply_raw(U, X, trans=False, compute=None, algo="auto", out=None, save=False):
    """Y = Q X (or Q^T X).  save=True (WY only) returns (Y, record) where the
    record holds the coefficients apply_bwd_raw(..., saved=record) uses."""
    _check_dev(U, X)
    X = _rows(X)
    param, io, comp = _cfg(X, compute)
    U = _param(U, param)
    N, n = X.shape
    h = U.shape[0]
    desc = L.make_desc(n, h, N, param, io, comp, algo)
    Y = torch.empty((N, n), dtype=io, device=X.device) if out is None else out
    op = L.HH_OP_APPLY_T if trans else L.HH_OP_APPLY
    ldu = max(n, U.stride(0) if h else n)
    if save:  # the record takes the place of the workspace (FP32 data: conversion space)
        rec = L.saved_record(op, desc, X.device)
        ws = L.workspace(op, desc, X.device) if io != comp else None
        L.check("hh_forward_save", L.lib().hh_forward_save(
            op, ctypes.byref(desc), L.ptr(U), ldu, None, L.ptr(X), L.ld(X), L.ptr(Y), L.ld(Y),
            L.ptr(rec), rec.numel(), L.ptr(ws), 0 if ws is None else ws.numel(), L.stream_of(X)))
        return Y, rec
    ws = L.workspace(op, desc, X.device)
    fn = L.lib().hh_apply_T if trans else L.lib().hh_apply
    L.check("hh_apply_T" if trans else "hh_apply",
            fn(ctypes.byref(desc), L.ptr(U), ldu, L.ptr(X), L.ld(X),
               L.ptr(Y), L.ld(Y), L.ptr(ws), ws.numel(), L.stream_of(X)))
    return Y


def sym_raw(U, lam, X, compute=None, algo="auto", out=None, save=False):
    """Y = Q diag(lam) Q^T X.  save=True (WY only) returns (Y, record)."""
    _check_dev(U, lam, X)
    X = _rows(X)
    param, io, comp = _cfg(X, compute)
    U, lam = _param(U, param), _param(lam, param)
    N, n = X.shape
    h = U.shape[0]
    desc = L.make_desc(n, h, N, param, io, comp, algo)
    Y = torch.empty((N, n), dtype=io, device=X.device) if out is None else out
    ldu = max(n, U.stride(0) if h else n)
    if save:  # the record takes the place of the workspace (FP32 data: conversion space)
        rec = L.saved_record(L.HH_OP_SYM, desc, X.device)
        ws = L.workspace(L.HH_OP_SYM, desc, X.device) if io != comp else None
        L.check("hh_forward_save", L.lib().hh_forward_save(
            L.HH_OP_SYM, ctypes.byref(desc), L.ptr(U), ldu, L.ptr(lam), L.ptr(X), L.ld(X),
            L.ptr(Y), L.ld(Y), L.ptr(rec), rec.numel(), L.ptr(ws), 0 if ws is None else ws.numel(),
            L.stream_of(X)))
        return Y, rec
    ws = L.workspace(L.HH_OP_SYM, desc, X.device)
    L.check("hh_sym_apply", L.lib().hh_sym_apply(
        ctypes.byref(desc), L.ptr(U), ldu, L.ptr(lam), L.ptr(X),
        L.ld(X), L.ptr(Y), L.ld(Y), L.ptr(ws), ws.numel(), L.stream_of(X)))
    return Y


def mahal_raw(U, lam, Xa, Xb, compute=None, algo="auto", save=False):
    """Distances d_j = sum_i lam_i ((Q^T (xa_j - xb_j))_i)^2.  save=True (fused
    algorithm) returns (d, record): the record holds each pair's h dot
    products, which mahal_bwd_raw(..., saved=record) reads instead of forming
    them again."""
    _check_dev(U, lam, Xa, Xb)
    Xa, Xb = _rows(Xa), _rows(Xb)
    param, io, comp = _cfg(Xa, compute)
    U, lam = _param(U, param), _param(lam, param)
    N, n = Xa.shape
    h = U.shape[0]
    desc = L.make_desc(n, h, N, param, io, comp, algo)
    d = torch.empty((N,), dtype=param, device=Xa.device)
    ws = L.workspace(L.HH_OP_MAHAL, desc, Xa.device)
    ldu = max(n, U.stride(0) if h else n)
    if not save:
        L.check("hh_mahalanobis", L.lib().hh_mahalanobis(
            ctypes.byref(desc), L.ptr(U), ldu, L.ptr(lam), L.ptr(Xa), L.ld(Xa), L.ptr(Xb), L.ld(Xb),
            L.ptr(d), L.ptr(ws), ws.numel(), L.stream_of(Xa)))
        return d
    nb = ctypes.c_size_t(0)
    L.check("hh_mahalanobis_saved_size", L.lib().hh_mahalanobis_saved_size(ctypes.byref(desc),
                                                                             ctypes.byref(nb)))
    rec = torch.empty((max(nb.value, 1),), dtype=torch.uint8, device=Xa.device)
    L.check("hh_mahalanobis_save", L.lib().hh_mahalanobis_save(
        ctypes.byref(desc), L.ptr(U), ldu, L.ptr(lam), L.ptr(Xa), L.ld(Xa), L.ptr(Xb), L.ld(Xb),
        L.ptr(d), L.ptr(rec), nb.value, L.ptr(ws), ws.numel(), L.stream_of(Xa)))
    return d, rec


def signed_raw(op, U, X, d_in=None, d_out=None, lam=None, Xb=None, compute=None, algo="auto",
               out=None):
    """The forward op ("apply", "apply_T", "sym" or "mahal") with diagonals on
    either side: diag(d_out) op(diag(d_in) X), or for "mahal" the distances of
    diag(d_in) (xa - xb).  Eq. 1's D Q is op "apply" with d_out = d, eq.
    thesbar's D Q diag(lam) Q^T D is "sym" with d_in = d_out = d.  Fused
    (FP32/FP64) algorithm only."""
    ops = {"apply": L.HH_OP_APPLY, "apply_T": L.HH_OP_APPLY_T, "sym": L.HH_OP_SYM,
           "mahal": L.HH_OP_MAHAL}
    hop = ops[op]
    _check_dev(U, X, *[t for t in (d_in, d_out, lam, Xb) if t is not None])
    X = _rows(X)
    param, io, comp = _cfg(X, compute)
    U = _param(U, param)
    N, n = X.shape
    h = U.shape[0]
    desc = L.make_desc(n, h, N, param, io, comp, algo)
    for name, t in (("d_in", d_in), ("d_out", d_out), ("lam", lam)):
        if t is not None and t.numel() != n:
            raise ValueError(f"{name} must hold n = {n} values, got {t.numel()}")
    d_in = None if d_in is None else _param(d_in, param)
    d_out = None if d_out is None else _param(d_out, param)
    lam = None if lam is None else _param(lam, param)
    if hop == L.HH_OP_MAHAL:
        Xb = _rows(Xb)
        Y = torch.empty((N,), dtype=param, device=X.device) if out is None else out
        ldy, ldb = 1, L.ld(Xb)
    else:
        Y = torch.empty((N, n), dtype=io, device=X.device) if out is None else out
        ldy, ldb = L.ld(Y), 0
    ws = L.workspace(hop, desc, X.device)
    L.check("hh_forward_signed", L.lib().hh_forward_signed(
        hop, ctypes.byref(desc), L.ptr(U), max(n, U.stride(0) if h else n), L.ptr(lam),
        L.ptr(d_in), L.ptr(d_out), L.ptr(X), L.ld(X), L.ptr(Xb), ldb, L.ptr(Y), ldy,
        L.ptr(ws), ws.numel(), L.stream_of(X)))
    return Y


def forward_noalloc_raw(op, U, X, lam=None, Xb=None, compute=None, algo="auto", out=None):
    """The forward op ("apply", "apply_T", "sym" or "mahal") through
    hh_forward_noalloc: no workspace is allocated (the library's static device
    scratch is used; calls that overlap on one GPU race).  Only the output is
    allocated here, unless ``out`` is given."""
    ops = {"apply": L.HH_OP_APPLY, "apply_T": L.HH_OP_APPLY_T, "sym": L.HH_OP_SYM,
           "mahal": L.HH_OP_MAHAL}
    hop = ops[op]
    _check_dev(U, X, *[t for t in (lam, Xb) if t is not None])
    X = _rows(X)
    param, io, comp = _cfg(X, compute)
    U = _param(U, param)
    lam = None if lam is None else _param(lam, param)
    N, n = X.shape
    h = U.shape[0]
    desc = L.make_desc(n, h, N, param, io, comp, algo)
    if hop == L.HH_OP_MAHAL:
        Xb = _rows(Xb)
        Y = torch.empty((N,), dtype=param, device=X.device) if out is None else out
        ldy, ldb = 0, L.ld(Xb)
    else:
        Y = torch.empty((N, n), dtype=io, device=X.device) if out is None else out
        ldy, ldb = L.ld(Y), 0
    L.check("hh_forward_noalloc", L.lib().hh_forward_noalloc(
        hop, ctypes.byref(desc), L.ptr(U), max(n, U.stride(0) if h else n), L.ptr(lam),
        L.ptr(X), L.ld(X), L.ptr(Xb), ldb, L.ptr(Y), ldy, L.stream_of(X)))
    return Y


def apply_bwd_raw(U, X, dY, trans=False, compute=None, algo="auto", need_dX=True, need_dU=True,
                  saved=None):
    """Gradients of Y = Q X (or Q^T X); saved: the forward's record (WY only)."""
    _check_dev(U, X, dY)
    X, dY = _rows(X), _rows(dY.to(X.dtype))
    param, io, comp = _cfg(X, compute)
    U = _param(U, param)
    N, n = X.shape
    h = U.shape[0]
    desc = L.make_desc(n, h, N, param, io, comp, algo)
    dX = torch.empty((N, n), dtype=io, device=X.device) if need_dX else None
    dU = torch.empty((h, n), dtype=param, device=X.device) if need_dU else None
    op = L.HH_OP_APPLY_T_BWD if trans else L.HH_OP_APPLY_BWD
    ws = L.workspace(op, desc, X.device)
    ldu = max(n, U.stride(0) if h else n)
    lddx = n if dX is None else L.ld(dX)
    if saved is not None:
        L.check("hh_backward_saved", L.lib().hh_backward_saved(
            op, ctypes.byref(desc), L.ptr(U), ldu, None, L.ptr(X), L.ld(X), L.ptr(saved),
            saved.numel(), L.ptr(dY), L.ld(dY), L.ptr(dX), lddx, L.ptr(dU), n, None,
            L.ptr(ws), ws.numel(), L.stream_of(X)))
        return dX, dU
    fn = L.lib().hh_apply_T_backward if trans else L.lib().hh_apply_backward
    L.check("hh_apply_T_backward" if trans else "hh_apply_backward",
            fn(ctypes.byref(desc), L.ptr(U), ldu, L.ptr(X), L.ld(X),
               L.ptr(dY), L.ld(dY), L.ptr(dX), lddx, L.ptr(dU), n,
               L.ptr(ws), ws.numel(), L.stream_of(X)))
    return dX, dU


def sym_bwd_raw(U, lam, X, dY, compute=None, algo="auto", need_dX=True, need_dU=True,
                need_dlam=True, saved=None):
    """Gradients of Y = Q diag(lam) Q^T X; saved: the forward's record (WY only)."""
    _check_dev(U, lam, X, dY)
    X, dY = _rows(X), _rows(dY.to(X.dtype))
    param, io, comp = _cfg(X, compute)
    U, lam = _param(U, param), _param(lam, param)
    N, n = X.shape
    h = U.shape[0]
    desc = L.make_desc(n, h, N, param, io, comp, algo)
    dX = torch.empty((N, n), dtype=io, device=X.device) if need_dX else None
    dU = torch.empty((h, n), dtype=param, device=X.device) if need_dU else None
    dlam = torch.empty((n,), dtype=param, device=X.device) if need_dlam else None
    ws = L.workspace(L.HH_OP_SYM_BWD, desc, X.device)
    ldu = max(n, U.stride(0) if h else n)
    lddx = n if dX is None else L.ld(dX)
    if saved is not None:
        L.check("hh_backward_saved", L.lib().hh_backward_saved(
            L.HH_OP_SYM_BWD, ctypes.byref(desc), L.ptr(U), ldu, L.ptr(lam), L.ptr(X), L.ld(X),
            L.ptr(saved), saved.numel(), L.ptr(dY), L.ld(dY), L.ptr(dX), lddx, L.ptr(dU), n,
            L.ptr(dlam), L.ptr(ws), ws.numel(), L.stream_of(X)))
        return dX, dU, dlam
    L.check("hh_sym_apply_backward", L.lib().hh_sym_apply_backward(
        ctypes.byref(desc), L.ptr(U), ldu, L.ptr(lam), L.ptr(X),
        L.ld(X), L.ptr(dY), L.ld(dY), L.ptr(dX), lddx, L.ptr(dU), n,
        L.ptr(dlam), L.ptr(ws), ws.numel(), L.stream_of(X)))
    return dX, dU, dlam


def mahal_bwd_raw(U, lam, Xa, Xb, dd, compute=None, algo="auto", need_dX=True, need_dU=True,
                  need_dlam=True, saved=None):
    """Gradients (dXa, dXb, dU, dlam) of sum_j dd_j d_j.  saved: the record of
    mahal_raw(..., save=True) on the same inputs."""
    _check_dev(U, lam, Xa, Xb, dd)
    Xa, Xb = _rows(Xa), _rows(Xb)
    param, io, comp = _cfg(Xa, compute)
    U, lam, dd = _param(U, param), _param(lam, param), _param(dd, param)
    N, n = Xa.shape
    h = U.shape[0]
    desc = L.make_desc(n, h, N, param, io, comp, algo)
    dXa = torch.empty((N, n), dtype=io, device=Xa.device) if need_dX else None
    dXb = torch.empty((N, n), dtype=io, device=Xa.device) if need_dX else None
    dU = torch.empty((h, n), dtype=param, device=Xa.device) if need_dU else None
    dlam = torch.empty((n,), dtype=param, device=Xa.device) if need_dlam else None
    ws = L.workspace(L.HH_OP_MAHAL_BWD, desc, Xa.device)
    ldu = max(n, U.stride(0) if h else n)
    if saved is None:
        L.check("hh_mahalanobis_backward", L.lib().hh_mahalanobis_backward(
            ctypes.byref(desc), L.ptr(U), ldu, L.ptr(lam), L.ptr(Xa), L.ld(Xa), L.ptr(Xb), L.ld(Xb),
            L.ptr(dd), L.ptr(dXa), L.ptr(dXb), n, L.ptr(dU), n, L.ptr(dlam), L.ptr(ws), ws.numel(),
            L.stream_of(Xa)))
    else:
        _check_dev(saved)
        L.check("hh_mahalanobis_backward_saved", L.lib().hh_mahalanobis_backward_saved(
            ctypes.byref(desc), L.ptr(U), ldu, L.ptr(lam), L.ptr(Xa), L.ld(Xa), L.ptr(Xb), L.ld(Xb),
            L.ptr(saved), saved.numel(), L.ptr(dd), L.ptr(dXa), L.ptr(dXb), n, L.ptr(dU), n,
            L.ptr(dlam), L.ptr(ws), ws.numel(), L.stream_of(Xa)))
    return dXa, dXb, dU, dlam


def signed_bwd_raw(op, U, X, dY, d_in=None, d_out=None, lam=None, Xb=None, compute=None,
                   algo="auto", need_dX=True, need_dU=True, need_dlam=True):
    """Gradients of <dY, signed_raw(op, U, X, d_in, d_out, lam, Xb)>: returns
    (dX, dU, dlam) for "apply", "apply_T" and "sym" (dlam None unless "sym"),
    (dXa, dXb, dU, dlam) for "mahal" (dY = the N distance weights).  A
    gradient whose need_* flag is False is neither computed nor allocated
    (None is returned in its place)."""
    ops = {"apply": L.HH_OP_APPLY_BWD, "apply_T": L.HH_OP_APPLY_T_BWD, "sym": L.HH_OP_SYM_BWD,
           "mahal": L.HH_OP_MAHAL_BWD}
    hop = ops[op]
    _check_dev(U, X, dY, *[t for t in (d_in, d_out, lam, Xb) if t is not None])
    X = _rows(X)
    param, io, comp = _cfg(X, compute)
    U = _param(U, param)
    N, n = X.shape
    h = U.shape[0]
    for name, t in (("d_in", d_in), ("d_out", d_out), ("lam", lam)):
        if t is not None and t.numel() != n:
            raise ValueError(f"{name} must hold n = {n} values, got {t.numel()}")
    d_in = None if d_in is None else _param(d_in, param)
    d_out = None if d_out is None else _param(d_out, param)
    lam = None if lam is None else _param(lam, param)
    mahal = hop == L.HH_OP_MAHAL_BWD
    if mahal:
        Xb = _rows(Xb)
        dY = _param(dY, param)
        lddy, ldb = 0, L.ld(Xb)
    else:
        dY = _rows(dY.to(X.dtype))
        lddy, ldb = L.ld(dY), 0
    desc = L.make_desc(n, h, N, param, io, comp, algo)
    dX = torch.empty((N, n), dtype=io, device=X.device) if need_dX else None
    dXb = torch.empty((N, n), dtype=io, device=X.device) if (mahal and need_dX) else None
    dU = torch.empty((h, n), dtype=param, device=X.device) if need_dU else None
    has_lam = hop in (L.HH_OP_SYM_BWD, L.HH_OP_MAHAL_BWD)
    dlam = torch.empty((n,), dtype=param, device=X.device) if (has_lam and need_dlam) else None
    ws = L.workspace(hop, desc, X.device)
    L.check("hh_backward_signed", L.lib().hh_backward_signed(
        hop, ctypes.byref(desc), L.ptr(U), max(n, U.stride(0) if h else n), L.ptr(lam),
        L.ptr(d_in), L.ptr(d_out), L.ptr(X), L.ld(X), L.ptr(Xb), ldb, L.ptr(dY), lddy,
        L.ptr(dX), L.ptr(dXb), n if dX is None else L.ld(dX), L.ptr(dU), n, L.ptr(dlam),
        L.ptr(ws), ws.numel(), L.stream_of(X)))
    return (dX, dXb, dU, dlam) if mahal else (dX, dU, dlam)


# --------------------------------------------------------------------------
# autograd
# --------------------------------------------------------------------------
class _Apply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, X, trans, compute, algo):
        ctx.cfg = (trans, compute, algo)
        rec = None
        if ctx.needs_input_grad[0] and is_wy(X, compute, algo):
            Y, rec = apply_raw(U, X, trans, compute, algo, save=True)
        else:
            Y = apply_raw(U, X, trans, compute, algo)
        ctx.save_for_backward(U, X, rec)
        return Y

    @staticmethod
    def backward(ctx, dY):
        U, X, rec = ctx.saved_tensors
        trans, compute, algo = ctx.cfg
        dX, dU = apply_bwd_raw(U, X, dY, trans, compute, algo,
                               need_dX=ctx.needs_input_grad[1], need_dU=ctx.needs_input_grad[0],
                               saved=rec)
        if dU is not None:
            dU = dU.to(U.dtype)
        return dU, dX, None, None, None


class _Sym(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, lam, X, compute, algo):
        ctx.cfg = (compute, algo)
        rec = None
        if (ctx.needs_input_grad[0] or ctx.needs_input_grad[1]) and is_wy(X, compute, algo):
            Y, rec = sym_raw(U, lam, X, compute, algo, save=True)
        else:
            Y = sym_raw(U, lam, X, compute, algo)
        ctx.save_for_backward(U, lam, X, rec)
        return Y

    @staticmethod
    def backward(ctx, dY):
        U, lam, X, rec = ctx.saved_tensors
        compute, algo = ctx.cfg
        dX, dU, dlam = sym_bwd_raw(U, lam, X, dY, compute, algo,
                                   need_dX=ctx.needs_input_grad[2],
                                   need_dU=ctx.needs_input_grad[0],
                                   need_dlam=ctx.needs_input_grad[1], saved=rec)
        if dU is not None:
            dU = dU.to(U.dtype)
        if dlam is not None:
            dlam = dlam.to(lam.dtype)
        return dU, dlam, dX, None, None


class _Mahal(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, lam, Xa, Xb, compute, algo):
        ctx.cfg = (compute, algo)
        ctx.save_for_backward(U, lam, Xa, Xb)
        ctx.rec = None
        comp = _cfg(Xa, compute)[2]
        fused = algo in ("auto", "fused", "fused_qr") and comp in (torch.float32, torch.float64)
        if fused and (ctx.needs_input_grad[0] or ctx.needs_input_grad[1]):
            # the forward keeps its dot products for the backward (h values per pair)
            d, ctx.rec = mahal_raw(U, lam, Xa, Xb, compute, algo, save=True)
            return d
        return mahal_raw(U, lam, Xa, Xb, compute, algo)

    @staticmethod
    def backward(ctx, dd):
        U, lam, Xa, Xb = ctx.saved_tensors
        compute, algo = ctx.cfg
        need_x = ctx.needs_input_grad[2] or ctx.needs_input_grad[3]
        dXa, dXb, dU, dlam = mahal_bwd_raw(U, lam, Xa, Xb, dd.contiguous(), compute, algo,
                                           need_dX=need_x, need_dU=ctx.needs_input_grad[0],
                                           need_dlam=ctx.needs_input_grad[1], saved=ctx.rec)
        ctx.rec = None
        if dU is not None:
            dU = dU.to(U.dtype)
        if dlam is not None:
            dlam = dlam.to(lam.dtype)
        return (dU, dlam, dXa if ctx.needs_input_grad[2] else None,
                dXb if ctx.needs_input_grad[3] else None, None, None)


class _Signed(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op, U, X, d_in, d_out, lam, Xb, compute, algo):
        ctx.cfg = (op, compute, algo)
        ctx.save_for_backward(U, X, d_in, d_out, lam, Xb)
        return signed_raw(op, U, X, d_in, d_out, lam, Xb, compute, algo)

    @staticmethod
    def backward(ctx, dY):
        U, X, d_in, d_out, lam, Xb = ctx.saved_tensors
        op, compute, algo = ctx.cfg
        need = ctx.needs_input_grad  # (op, U, X, d_in, d_out, lam, Xb, compute, algo)
        r = signed_bwd_raw(op, U, X, dY.contiguous(), d_in, d_out, lam, Xb, compute, algo,
                           need_dX=need[2] or need[6], need_dU=need[1],
                           need_dlam=lam is not None and need[5])
        if op == "mahal":
            dX, dXb, dU, dlam = r
        else:
            (dX, dU, dlam), dXb = r, None
        if dU is not None:
            dU = dU.to(U.dtype)
        if dlam is not None:
            dlam = dlam.to(lam.dtype)
        return (None, dU, dX if need[2] else None, None, None, dlam,
                dXb if need[6] else None, None, None)


def signed(op, U, X, *, d_in=None, d_out=None, lam=None, Xb=None, compute=None, algo="auto"):
    """diag(d_out) op(diag(d_in) X) with gradients to U, X, lam and Xb (the
    diagonals are fixed signs, not differentiated: a diagonal that requires a
    gradient is rejected); op as in signed_raw."""
    for name, t in (("d_in", d_in), ("d_out", d_out)):
        if t is not None and t.requires_grad:
            raise ValueError(f"{name} is a fixed diagonal and has no gradient; pass {name}.detach()")
    return _Signed.apply(op, U, X, d_in, d_out, lam, Xb, compute, algo)


def apply(U, X, *, compute=None, algo="auto"):
    """Y = Q X with Q = H_1 ... H_h (rows of the result are Q x_j)."""
    return _Apply.apply(U, X, False, compute, algo)


def apply_T(U, X, *, compute=None, algo="auto"):
    """Y = Q^T X = H_h ... H_1 X."""
    return _Apply.apply(U, X, True, compute, algo)


def sym_apply(U, lam, X, *, compute=None, algo="auto"):
    """Y = Q diag(lam) Q^T X."""
    return _Sym.apply(U, lam, X, compute, algo)


def mahalanobis(U, lam, Xa, Xb, *, compute=None, algo="auto"):
    """d_j = sum_i lam_i ((Q^T (xa_j - xb_j))_i)^2."""
    return _Mahal.apply(U, lam, Xa, Xb, compute, algo)


# --------------------------------------------------------------------------
# orthonormal factorisation front-end
# --------------------------------------------------------------------------
_FACTOR = {"constrained": L.HH_FACTOR_CONSTRAINED, "unconstrained": L.HH_FACTOR_UNCONSTRAINED,
           "qr": L.HH_FACTOR_QR}


def factor_orthonormal(U, h, method="unconstrained"):
    """Reflectors approximating the orthonormal (n, n) matrix U (math
    orientation, device tensor): "constrained" (Result 1), "unconstrained"
    (Result 2) or "qr" (Result 3).  Returns (R, d, z): R (h, n) float64 in the
    library's reflector layout (row k = u_k, Q = H_1 ... H_h approximates U,
    or U ~ Q diag(d) for "qr"), d (n,) the sign diagonal (ones for the eigen
    methods), z (n,) the eigenvalues of U + U^T ascending (eigen methods;
    None for "qr")."""
    _check_dev(U)
    if U.dim() != 2 or U.shape[0] != U.shape[1]:
        raise ValueError("U must be square")
    n = U.shape[0]
    Ut = U.to(torch.float64).t().contiguous()  # column-major: (column j) = row j of Ut
    m = _FACTOR[method]
    nb = ctypes.c_size_t(0)
    L.check("hh_factor_workspace_size", L.lib().hh_factor_workspace_size(m, n, h, ctypes.byref(nb)))
    ws = torch.empty((max(nb.value, 1),), dtype=torch.uint8, device=U.device)
    R = torch.empty((h, n), dtype=torch.float64, device=U.device)
    d = torch.empty((n,), dtype=torch.float64, device=U.device)
    z = None if method == "qr" else torch.empty((n,), dtype=torch.float64, device=U.device)
    L.check("hh_factor_orthonormal", L.lib().hh_factor_orthonormal(
        m, n, h, L.ptr(Ut), n, L.ptr(R) if h else None, n, L.ptr(d), L.ptr(z), L.ptr(ws),
        ws.numel(), L.stream_of(Ut)))
    return R, d, z


def shf(S, h, K=30, spectrum_update=True):
    """Symmetric Householder Factorisation of the symmetric (n, n) device
    tensor S (Algorithm 1; SHF-SU when spectrum_update): returns (R, sbar, d,
    err) with R (h, n) float64 reflectors (row k = u_k), so that
    Sbar = D Q diag(sbar) Q^T D with Q = H_1 ... H_h (apply it with
    signed("sym", R, X, d_in=d, d_out=d, lam=sbar)), and err (K + 1,) the
    squared Frobenius errors after the initialisation and each sweep."""
    _check_dev(S)
    if S.dim() != 2 or S.shape[0] != S.shape[1]:
        raise ValueError("S must be square")
    n = S.shape[0]
    St = S.to(torch.float64).contiguous()  # symmetric: row- and column-major agree
    nb = ctypes.c_size_t(0)
    L.check("hh_shf_workspace_size", L.lib().hh_shf_workspace_size(n, h, K, ctypes.byref(nb)))
    ws = torch.empty((nb.value,), dtype=torch.uint8, device=S.device)
    R = torch.empty((h, n), dtype=torch.float64, device=S.device)
    sbar = torch.empty((n,), dtype=torch.float64, device=S.device)
    d = torch.empty((n,), dtype=torch.float64, device=S.device)
    err = torch.empty((K + 1,), dtype=torch.float64, device=S.device)
    L.check("hh_shf", L.lib().hh_shf(n, h, K, 1 if spectrum_update else 0, L.ptr(St), n,
                                     L.ptr(R) if h else None, n, L.ptr(sbar), L.ptr(d),
                                     L.ptr(err), L.ptr(ws), ws.numel(), L.stream_of(St)))
    return R, sbar, d, err


def knn_raw(Zq, Zd, k):
    """k nearest database rows of Zd (Nd, n) for every query row of Zq (Nq, n)
    in squared Euclidean distance (FP32 device tensors of transformed
    vectors): returns (dist (Nq, k) float32 ascending, idx (Nq, k) int64)."""
    _check_dev(Zq, Zd)
    Zq, Zd = _rows(Zq.to(torch.float32)), _rows(Zd.to(torch.float32))
    Nq, n = Zq.shape
    Nd = Zd.shape[0]
    dist = torch.empty((Nq, k), dtype=torch.float32, device=Zq.device)
    idx = torch.empty((Nq, k), dtype=torch.int64, device=Zq.device)
    nb = ctypes.c_size_t(0)
    L.check("hh_knn_workspace_size", L.lib().hh_knn_workspace_size(n, Nq, Nd, k, ctypes.byref(nb)))
    ws = torch.empty((max(nb.value, 1),), dtype=torch.uint8, device=Zq.device)
    L.check("hh_knn", L.lib().hh_knn(n, Nq, Nd, k, L.ptr(Zq), L.ld(Zq), L.ptr(Zd), L.ld(Zd),
                                     L.ptr(dist), L.ptr(idx), L.ptr(ws), ws.numel(), L.stream_of(Zq)))
    return dist, idx


def knn(U, lam, Xq, Xd, k):
    """k nearest neighbours in the learned metric d(x, y) = sum_i lam_i
    ((Q^T (x - y))_i)^2 (Sec. IV-C): both sets are transformed by
    L = diag(sqrt(lam)) Q^T on the fused kernels (one pass each), then
    knn_raw runs on the transformed vectors."""
    sq = torch.sqrt(lam.to(torch.float32))
    Zq = signed_raw("apply_T", U, Xq.to(torch.float32), d_out=sq)
    Zd = signed_raw("apply_T", U, Xd.to(torch.float32), d_out=sq)
    return knn_raw(Zq, Zd, k)
