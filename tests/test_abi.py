"""Host-side checks of the C ABI: the library loads, exports every symbol that
include/hh.h declares, and validates arguments before touching a device.
No compute call is made here."""
import ctypes
import os
import re

import pytest

import paper_1811_07624_amd as P
from paper_1811_07624_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"HH_API[^;(]*?\b(hh_\w+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("hh_apply", "hh_apply_T", "hh_sym_apply", "hh_mahalanobis", "hh_apply_backward",
              "hh_apply_T_backward", "hh_sym_apply_backward", "hh_mahalanobis_backward",
              "hh_workspace_size"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    lib = P.lib()
    for s in declared_symbols():
        assert hasattr(lib, s), s
    assert set(L.EXPORTS) <= set(declared_symbols())


def _desc(n=8, h=2, N=4, p=L.HH_F32, io=L.HH_F32, c=L.HH_F32, algo=L.HH_ALGO_AUTO):
    return L.HHDesc(n, h, N, p, io, c, algo)


def _apply(desc, U=1, ldu=8, X=2, ldx=8, Y=3, ldy=8, ws=None, wsb=0):
    # fake non-null pointers: every failure below is caught before any launch
    v = ctypes.c_void_p
    return P.lib().hh_apply(ctypes.byref(desc), v(U), ldu, v(X), ldx, v(Y), ldy, v(ws) if ws else None,
                            wsb, None)


@pytest.mark.parametrize("field,value", [("n", 0), ("h", -1), ("N", -5)])
def test_invalid_shapes(field, value):
    d = _desc()
    setattr(d, field, value)
    assert _apply(d) == L.HH_ERR_INVALID_ARG
    assert P.lib().hh_last_error().decode() != ""


def test_invalid_leading_dimension():
    assert _apply(_desc(), ldx=7) == L.HH_ERR_INVALID_ARG
    assert b"ldx" in P.lib().hh_last_error()
    assert _apply(_desc(), ldy=3) == L.HH_ERR_INVALID_ARG


def test_unsupported_combinations():
    # FUSED with mixed dtypes
    assert _apply(_desc(p=L.HH_F64)) == L.HH_ERR_UNSUPPORTED
    # WY with F64 parameters
    assert _apply(_desc(p=L.HH_F64, io=L.HH_BF16, c=L.HH_BF16)) == L.HH_ERR_UNSUPPORTED
    # FUSED forced on a 16-bit compute type
    assert _apply(_desc(c=L.HH_BF16, algo=L.HH_ALGO_FUSED)) == L.HH_ERR_UNSUPPORTED
    # WY data: the compute type or F32 (converted), not the other 16-bit type
    assert _apply(_desc(n=64, h=4, p=L.HH_F32, io=L.HH_F16, c=L.HH_BF16)) == L.HH_ERR_UNSUPPORTED
    # F32 data on WY: n must be a multiple of 8; a missing workspace is caught
    # before anything is enqueued
    assert _apply(_desc(n=60, h=4, p=L.HH_F32, io=L.HH_F32, c=L.HH_BF16), ldu=60, ldx=60,
                  ldy=60) == L.HH_ERR_UNSUPPORTED
    assert _apply(_desc(n=64, h=4, p=L.HH_F32, io=L.HH_F32, c=L.HH_BF16), ldu=64, ldx=64,
                  ldy=64) == L.HH_ERR_INVALID_ARG
    # fused kernels cover n <= 8192 (FP32)
    assert _apply(_desc(n=8193), ldu=8193, ldx=8193, ldy=8193) == L.HH_ERR_UNSUPPORTED


def test_null_pointers_and_workspace():
    d = _desc()
    nb = ctypes.c_size_t(0)
    assert P.lib().hh_workspace_size(L.HH_OP_APPLY, ctypes.byref(d), ctypes.byref(nb)) == L.HH_OK
    assert nb.value > 0
    assert _apply(d, X=0, ws=16, wsb=nb.value) == L.HH_ERR_INVALID_ARG
    assert _apply(d, ws=16, wsb=nb.value - 1) == L.HH_ERR_WORKSPACE
    assert _apply(d, ws=None, wsb=0) in (L.HH_ERR_INVALID_ARG, L.HH_ERR_WORKSPACE)


def test_in_place_needs_equal_ld():
    d = _desc()
    nb = ctypes.c_size_t(0)
    P.lib().hh_workspace_size(L.HH_OP_APPLY, ctypes.byref(d), ctypes.byref(nb))
    assert _apply(d, X=64, Y=64, ldx=8, ldy=16, ws=16, wsb=nb.value) == L.HH_ERR_INVALID_ARG


def test_n_zero_batch_is_noop():
    d = _desc(N=0)
    # N = 0: nothing is enqueued, so fake pointers are never touched
    assert _apply(d, X=0, Y=0, ws=None, wsb=0) == L.HH_OK


def test_workspace_size_all_ops():
    for op in range(8):
        for (p, io, c) in [(L.HH_F32, L.HH_F32, L.HH_F32), (L.HH_F64, L.HH_F64, L.HH_F64)]:
            d = _desc(n=512, h=9, N=1000, p=p, io=io, c=c)
            nb = ctypes.c_size_t(0)
            assert P.lib().hh_workspace_size(op, ctypes.byref(d), ctypes.byref(nb)) == L.HH_OK


def test_status_strings():
    for s in range(5):
        assert P.lib().hh_status_string(s)


def _wy_desc(n=256, h=12, N=100, c=L.HH_BF16):
    return L.HHDesc(n, h, N, L.HH_F32, c, c, L.HH_ALGO_AUTO)


def test_saved_size():
    nb = ctypes.c_size_t(0)
    lib = P.lib()
    # m = h rounded up to 64 (128 for h > 64), doubled for the symmetric form;
    # row stride = N rounded up to 32
    for (n, h, N, op, m) in [(256, 12, 100, L.HH_OP_APPLY, 64), (256, 12, 100, L.HH_OP_APPLY_T, 64),
                             (256, 12, 100, L.HH_OP_SYM, 128), (8192, 100, 1, L.HH_OP_SYM, 256),
                             (1024, 64, 0, L.HH_OP_APPLY, 64)]:
        d = _wy_desc(n, h, N)
        assert lib.hh_saved_size(op, ctypes.byref(d), ctypes.byref(nb)) == L.HH_OK
        # coefficient rows first, then the setup (256-byte aligned parts)
        coef = m * max(32, (N + 31) // 32 * 32) * 2
        assert nb.value > coef and nb.value % 256 == 0
        d2 = _wy_desc(n, h, N + 64)
        nb2 = ctypes.c_size_t(0)
        lib.hh_saved_size(op, ctypes.byref(d2), ctypes.byref(nb2))
        coef2 = m * ((N + 64 + 31) // 32 * 32) * 2
        assert nb2.value - nb.value == -(-coef2 // 256) * 256 - (-(-coef // 256) * 256)
    d = _wy_desc()
    assert lib.hh_saved_size(L.HH_OP_MAHAL, ctypes.byref(d), ctypes.byref(nb)) == L.HH_ERR_INVALID_ARG
    assert lib.hh_saved_size(L.HH_OP_APPLY_BWD, ctypes.byref(d), ctypes.byref(nb)) == L.HH_ERR_INVALID_ARG
    # the fused backward keeps no coefficients
    assert lib.hh_saved_size(L.HH_OP_APPLY, ctypes.byref(_desc()), ctypes.byref(nb)) == L.HH_ERR_UNSUPPORTED


def test_saved_record_validation():
    # fake, 16-byte aligned pointers: every failure below is caught before any launch
    v = ctypes.c_void_p
    lib = P.lib()
    d = _wy_desc()
    nb, ws = ctypes.c_size_t(0), ctypes.c_size_t(0)
    lib.hh_saved_size(L.HH_OP_APPLY, ctypes.byref(d), ctypes.byref(nb))
    lib.hh_workspace_size(L.HH_OP_APPLY, ctypes.byref(d), ctypes.byref(ws))

    def fwd(op=L.HH_OP_APPLY, saved=4096, sb=nb.value, desc=d):
        return lib.hh_forward_save(op, ctypes.byref(desc), v(1024), 256, None, v(2048), 256, v(3072),
                                   256, v(saved) if saved else None, sb, v(8192), ws.value, None)
    assert fwd(saved=0) == L.HH_ERR_INVALID_ARG
    assert fwd(sb=nb.value - 1) == L.HH_ERR_INVALID_ARG
    assert fwd(saved=4100) == L.HH_ERR_INVALID_ARG            # not 16-byte aligned
    assert fwd(op=L.HH_OP_MAHAL) == L.HH_ERR_INVALID_ARG
    assert fwd(desc=_desc()) == L.HH_ERR_UNSUPPORTED           # fused path

    def bwd(op=L.HH_OP_APPLY_BWD, saved=4096, sb=nb.value, desc=d):
        return lib.hh_backward_saved(op, ctypes.byref(desc), v(1024), 256, None, v(2048), 256,
                                     v(saved) if saved else None, sb, v(3072), 256, v(5120), 256,
                                     v(6144), 256, None, v(8192), 1 << 40, None)
    assert bwd(saved=0) == L.HH_ERR_INVALID_ARG
    assert bwd(op=L.HH_OP_APPLY) == L.HH_ERR_INVALID_ARG
    assert bwd(sb=nb.value - 1) == L.HH_ERR_INVALID_ARG
    assert bwd(saved=4104) == L.HH_ERR_INVALID_ARG
    assert bwd(desc=_desc()) == L.HH_ERR_UNSUPPORTED


def test_signed_validation():
    # fake, aligned pointers: every failure below is caught before any launch
    v = ctypes.c_void_p
    lib = P.lib()

    def fwd(op=L.HH_OP_APPLY, desc=None, d_in=0, d_out=0, lam=None, ld=8):
        dp = ctypes.byref(desc if desc is not None else _desc()) if desc is not False else None
        return lib.hh_forward_signed(op, dp, v(1024), ld, v(lam) if lam else None,
                                     v(d_in) if d_in else None, v(d_out) if d_out else None,
                                     v(2048), ld, v(4096), ld, v(3072), ld, v(8192), 1 << 20, None)
    assert fwd(op=L.HH_OP_APPLY_BWD, d_in=5120) == L.HH_ERR_INVALID_ARG
    assert fwd(desc=False, d_in=5120) == L.HH_ERR_INVALID_ARG
    assert fwd(d_in=5122) == L.HH_ERR_INVALID_ARG                     # not aligned to 4 bytes
    assert fwd(d_out=5122) == L.HH_ERR_INVALID_ARG
    assert fwd(desc=_desc(p=L.HH_F64, io=L.HH_F64, c=L.HH_F64), d_in=5124) == L.HH_ERR_INVALID_ARG
    assert fwd(op=L.HH_OP_MAHAL, d_out=5120, lam=6144) == L.HH_ERR_INVALID_ARG  # a distance has no output side
    assert fwd(desc=_wy_desc(), d_in=5120, ld=256) == L.HH_ERR_UNSUPPORTED      # fused path only
    assert fwd(desc=_wy_desc(), d_out=5120, ld=256) == L.HH_ERR_UNSUPPORTED


def test_signed_backward_validation():
    v = ctypes.c_void_p
    lib = P.lib()

    def bwd(op=L.HH_OP_APPLY_BWD, desc=None, d_in=0, d_out=0, ld=8):
        dp = ctypes.byref(desc if desc is not None else _desc())
        return lib.hh_backward_signed(op, dp, v(1024), ld, v(6144), v(d_in) if d_in else None,
                                      v(d_out) if d_out else None, v(2048), ld, v(4096), ld,
                                      v(3072), ld, v(5120), v(7168), ld, v(9216), ld, v(10240),
                                      v(8192), 1 << 20, None)
    assert bwd(op=L.HH_OP_APPLY, d_in=12288) == L.HH_ERR_INVALID_ARG
    assert bwd(d_in=12290) == L.HH_ERR_INVALID_ARG                    # not aligned to 4 bytes
    assert bwd(op=L.HH_OP_MAHAL_BWD, d_out=12288) == L.HH_ERR_INVALID_ARG
    assert bwd(desc=_wy_desc(), d_in=12288, ld=256) == L.HH_ERR_UNSUPPORTED


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No fallback: without libhh.so every entry point raises instead of
    computing anything on the host."""
    import torch
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "libhh.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(ImportError):
        L.lib()
    U = torch.zeros((2, 8))
    X = torch.zeros((4, 8))
    with pytest.raises((ImportError, ValueError)):
        P.apply_raw(U, X)


def test_version():
    v = P.lib().hh_version()
    assert v >= 300 and v < 10000  # 0.x.y with the saved record, FP32 data on the WY path and diagonals


def test_signed_rejects_differentiable_diagonal():
    """The diagonals of P.signed are fixed signs: one that requires a gradient
    is refused before anything runs (it would otherwise get none silently)."""
    import torch
    U = torch.zeros((2, 8))
    X = torch.zeros((4, 8))
    d = torch.ones(8, requires_grad=True)
    with pytest.raises(ValueError, match="fixed diagonal"):
        P.signed("apply", U, X, d_in=d)
    with pytest.raises(ValueError, match="fixed diagonal"):
        P.signed("apply", U, X, d_out=d)


def test_noalloc_validation():
    """hh_forward_noalloc refuses, on the host and before any device call,
    backward ops, bad descriptors and calls whose workspace exceeds the static
    scratch (fake pointers: nothing is dereferenced)."""
    v = ctypes.c_void_p
    lib = P.lib()

    def call(op, desc):
        return lib.hh_forward_noalloc(op, ctypes.byref(desc), v(1024), desc.n, v(6144), v(2048),
                                      desc.n, v(4096), desc.n, v(3072), desc.n, None)
    assert call(L.HH_OP_APPLY_BWD, _desc()) == L.HH_ERR_INVALID_ARG
    assert call(L.HH_OP_APPLY, _desc(n=0)) == L.HH_ERR_INVALID_ARG
    assert call(L.HH_OP_MAHAL, _wy_desc()) == L.HH_ERR_UNSUPPORTED
    big = L.HHDesc(4096, 64, 4096, L.HH_F32, L.HH_F32, L.HH_BF16, L.HH_ALGO_AUTO)  # 64 MiB copies
    assert call(L.HH_OP_APPLY, big) == L.HH_ERR_WORKSPACE
    assert b"static scratch" in lib.hh_last_error()


def test_factor_validation():
    """The front-end refuses bad arguments on the host before any device call."""
    v = ctypes.c_void_p
    lib = P.lib()
    nb = ctypes.c_size_t(0)
    assert lib.hh_factor_workspace_size(L.HH_FACTOR_QR, 64, 63, ctypes.byref(nb)) == L.HH_OK
    assert nb.value >= 64 * 64 * 8
    assert lib.hh_factor_workspace_size(L.HH_FACTOR_QR, 64, 64, ctypes.byref(nb)) == L.HH_ERR_INVALID_ARG
    assert lib.hh_factor_workspace_size(7, 64, 4, ctypes.byref(nb)) == L.HH_ERR_INVALID_ARG
    assert lib.hh_factor_workspace_size(L.HH_FACTOR_CONSTRAINED, 2048, 4, ctypes.byref(nb)) == \
        L.HH_ERR_UNSUPPORTED
    assert lib.hh_factor_workspace_size(L.HH_FACTOR_CONSTRAINED, 0, 4, ctypes.byref(nb)) == \
        L.HH_ERR_INVALID_ARG

    def call(n=16, h=4, U=1024, ldu=16, R=2048, ldr=16, ws=4096, wsb=1 << 20):
        return lib.hh_factor_orthonormal(L.HH_FACTOR_UNCONSTRAINED, n, h, v(U) if U else None, ldu,
                                         v(R) if R else None, ldr, None, None,
                                         v(ws) if ws else None, wsb, None)
    assert call(U=0) == L.HH_ERR_INVALID_ARG
    assert call(ldu=15) == L.HH_ERR_INVALID_ARG
    assert call(R=0) == L.HH_ERR_INVALID_ARG
    assert call(ldr=3) == L.HH_ERR_INVALID_ARG
    assert call(ws=0) == L.HH_ERR_INVALID_ARG
    assert call(wsb=16) == L.HH_ERR_WORKSPACE


def test_shf_validation():
    v = ctypes.c_void_p
    lib = P.lib()
    nb = ctypes.c_size_t(0)
    assert lib.hh_shf_workspace_size(128, 16, 30, ctypes.byref(nb)) == L.HH_OK
    assert nb.value >= 7 * 128 * 128 * 8
    assert lib.hh_shf_workspace_size(513, 4, 3, ctypes.byref(nb)) == L.HH_ERR_UNSUPPORTED
    assert lib.hh_shf_workspace_size(16, -1, 3, ctypes.byref(nb)) == L.HH_ERR_INVALID_ARG

    def call(S=1024, lds=16, R=2048, ws=4096, wsb=1 << 22):
        return lib.hh_shf(16, 2, 3, 1, v(S) if S else None, lds, v(R) if R else None, 16, v(6144),
                          v(7168), None, v(ws) if ws else None, wsb, None)
    assert call(S=0) == L.HH_ERR_INVALID_ARG
    assert call(lds=8) == L.HH_ERR_INVALID_ARG
    assert call(R=0) == L.HH_ERR_INVALID_ARG
    assert call(wsb=64) == L.HH_ERR_WORKSPACE


def test_knn_validation():
    v = ctypes.c_void_p
    lib = P.lib()

    def call(n=8, Nq=4, Nd=10, k=3, ldq=8, ldd=8, ptr=1024, wsb=1 << 20):
        p = v(ptr) if ptr else None
        return lib.hh_knn(n, Nq, Nd, k, p, ldq, p, ldd, p, p, p, wsb, None)
    assert call(wsb=8) == L.HH_ERR_WORKSPACE
    assert call(k=0) == L.HH_ERR_INVALID_ARG
    assert call(k=11) == L.HH_ERR_INVALID_ARG      # k > Nd
    assert call(k=33, Nd=100) == L.HH_ERR_UNSUPPORTED
    assert call(n=225, ldq=225, ldd=225) == L.HH_ERR_UNSUPPORTED
    assert call(ldq=7) == L.HH_ERR_INVALID_ARG
    assert call(ptr=0) == L.HH_ERR_INVALID_ARG
    assert call(Nq=0, ptr=0) == L.HH_OK


def test_mahal_record_validation():
    """The distance record (fused path): its size, and the checks that fail
    before anything is enqueued (fake pointers: nothing is dereferenced)."""
    v = ctypes.c_void_p
    lib = P.lib()
    nb = ctypes.c_size_t(0)
    d = _desc(n=8, h=3, N=100)
    assert lib.hh_mahalanobis_saved_size(ctypes.byref(d), ctypes.byref(nb)) == L.HH_OK
    assert nb.value == -(-4 * 100 * 4 // 256) * 256  # N rows of h = 3 padded to 4 FP32 values
    d64 = _desc(n=8, h=3, N=100, p=L.HH_F64, io=L.HH_F64, c=L.HH_F64)
    assert lib.hh_mahalanobis_saved_size(ctypes.byref(d64), ctypes.byref(nb)) == L.HH_OK
    assert nb.value == -(-4 * 100 * 8 // 256) * 256  # rows of 3 FP64 values padded to 4
    assert lib.hh_mahalanobis_saved_size(ctypes.byref(d), None) == L.HH_ERR_INVALID_ARG
    assert lib.hh_mahalanobis_saved_size(ctypes.byref(_wy_desc()), ctypes.byref(nb)) == L.HH_ERR_UNSUPPORTED
    lib.hh_mahalanobis_saved_size(ctypes.byref(d), ctypes.byref(nb))

    def fwd(saved=4096, sb=nb.value, desc=d):
        return lib.hh_mahalanobis_save(ctypes.byref(desc), v(1024), 8, v(2048), v(3072), 8, v(5120), 8,
                                       v(6144), v(saved) if saved else None, sb, v(8192), 1 << 40, None)
    assert fwd(saved=0) == L.HH_ERR_INVALID_ARG
    assert fwd(sb=nb.value - 1) == L.HH_ERR_WORKSPACE
    assert fwd(desc=_wy_desc()) == L.HH_ERR_UNSUPPORTED

    def bwd(saved=4096, sb=nb.value, desc=d):
        return lib.hh_mahalanobis_backward_saved(ctypes.byref(desc), v(1024), 8, v(2048), v(3072), 8,
                                                 v(5120), 8, v(saved) if saved else None, sb, v(6144),
                                                 v(7168), v(9216), 8, v(10240), 8, v(11264), v(12288),
                                                 1 << 40, None)
    assert bwd(saved=0) == L.HH_ERR_INVALID_ARG
    assert bwd(sb=nb.value - 1) == L.HH_ERR_WORKSPACE
    assert bwd(desc=_wy_desc()) == L.HH_ERR_UNSUPPORTED
