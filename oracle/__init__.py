"""FP64 CPU oracle for the Householder-reflector hot path.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  It shares no code
with the HIP implementation.  The reflector arithmetic lives in
``hh_oracle.c`` (plain C, double precision, straightforward loops) and is
reached through ctypes; the only arithmetic in this module is the elementwise
diagonal products of ``signed`` / ``signed_bwd`` (numpy, FP64), written out as
the products of diagonal matrices they are.

Array conventions (numpy, C-contiguous float64):
  U   : (h, n)  row k is the reflector vector u_k  (column k of the n x h matrix)
  X   : (N, n)  row j is vector j of the batch     (column j of the n x N matrix)
  lam : (n,)
All functions take the raw (un-normalised) U; H_k = I - 2 uh_k uh_k^T with
uh_k = u_k/||u_k|| (eq. 2), and Q = H_1 ... H_h (product order of eq. 1 read
as in Result 3, eq. theU2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hh_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile hh_oracle.c into liboracle.so with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
             "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int64
    sigs = {
        "orc_normalize": [I, I, P, I, P, P],
        "orc_apply": [I, I, P, I, ctypes.c_int, P, I, I, P, I],
        "orc_dense_Q": [I, I, P, I, P],
        "orc_sym": [I, I, P, I, P, P, I, I, P, I],
        "orc_mahal": [I, I, P, I, P, P, I, P, I, I, P],
        "orc_apply_bwd": [I, I, P, I, ctypes.c_int, P, I, P, I, I, P, I, P, I],
        "orc_sym_bwd": [I, I, P, I, P, P, I, P, I, I, P, I, P, I, P],
        "orc_mahal_bwd": [I, I, P, I, P, P, I, P, I, P, I, P, P, I, P, I, P],
        "orc_householder_qr": [I, P, I, P, P],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = None
    lib.orc_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _shape_U(U):
    U = _f64(U)
    if U.ndim != 2:
        raise ValueError("U must be (h, n)")
    return U, U.shape[1], U.shape[0]


def num_threads() -> int:
    return int(_load().orc_num_threads())


def normalize(U):
    """uh_k = u_k/||u_k|| (eq. 2); zero rows stay zero.  Returns (Uh, norms)."""
    U, n, h = _shape_U(U)
    Uh = np.zeros((h, n))
    nrm = np.zeros(h)
    _load().orc_normalize(n, h, _p(U), n, _p(Uh), _p(nrm))
    return Uh, nrm


def apply(U, X, trans: bool = False):
    """Y = Q X (trans=False) or Q^T X (trans=True); X is (N, n)."""
    U, n, h = _shape_U(U)
    X = _f64(X)
    N = X.shape[0]
    assert X.shape[1] == n
    Y = np.empty_like(X)
    _load().orc_apply(n, h, _p(U), n, int(bool(trans)), _p(X), n, N, _p(Y), n)
    return Y


def dense_Q(U):
    """Explicit Q = H_1 ... H_h (n x n, math orientation), small n only."""
    U, n, h = _shape_U(U)
    Q = np.empty((n, n))
    _load().orc_dense_Q(n, h, _p(U), n, _p(Q))
    return Q.T.copy()  # column-major buffer -> math matrix


def sym(U, lam, X):
    """Y = Q diag(lam) Q^T X (Sec. III-A, eq. thesbar with D = I)."""
    U, n, h = _shape_U(U)
    lam = _f64(lam)
    X = _f64(X)
    N = X.shape[0]
    Y = np.empty_like(X)
    _load().orc_sym(n, h, _p(U), n, _p(lam), _p(X), n, N, _p(Y), n)
    return Y


def mahal(U, lam, Xa, Xb):
    """d_j = sum_i lam_i ((Q^T (xa_j - xb_j))_i)^2 (Sec. IV-C)."""
    U, n, h = _shape_U(U)
    lam, Xa, Xb = _f64(lam), _f64(Xa), _f64(Xb)
    N = Xa.shape[0]
    d = np.empty(N)
    _load().orc_mahal(n, h, _p(U), n, _p(lam), _p(Xa), n, _p(Xb), n, N, _p(d))
    return d


def signed(op, U, X, d_in=None, d_out=None, lam=None, Xb=None):
    """A forward op with diagonal matrices on either side, written out as
    products: diag(d_out) op(diag(d_in) X) for op "apply" (Q), "apply_T" (Q^T)
    and "sym" (Q diag(lam) Q^T); for "mahal" the distances of diag(d_in)(xa - xb).
    Eq. 1 puts D = diag(d) on the left of the reflector product (d_out = d with
    "apply"), Result 3 on its right (d_in = d), eq. thesbar on both sides of the
    symmetric form (d_in = d_out = d).  Rows of X are vectors, so diag(d) X is
    the columnwise product X * d."""
    X = _f64(X)
    n = X.shape[1]
    din = np.ones(n) if d_in is None else _f64(d_in)
    dout = np.ones(n) if d_out is None else _f64(d_out)
    if op == "mahal":
        assert d_out is None
        return mahal(U, lam, X * din, _f64(Xb) * din)
    if op == "apply":
        Y = apply(U, X * din)
    elif op == "apply_T":
        Y = apply(U, X * din, trans=True)
    elif op == "sym":
        Y = sym(U, lam, X * din)
    else:
        raise ValueError(op)
    return Y * dout


def signed_bwd(op, U, X, dY, d_in=None, d_out=None, lam=None, Xb=None):
    """Gradients of L = <dY, signed(op, U, X, d_in, d_out, lam, Xb)> by the
    chain rule through the two diagonal products: the plain op's gradients at
    X' = diag(d_in) X with upstream diag(d_out) dY, and dX = diag(d_in) dX'.
    Returns (dX, dU, dlam) (dlam None unless "sym"), or for "mahal" (dY = the
    N distance weights) (dXa, dXb, dU, dlam)."""
    X = _f64(X)
    n = X.shape[1]
    din = np.ones(n) if d_in is None else _f64(d_in)
    dout = np.ones(n) if d_out is None else _f64(d_out)
    if op == "mahal":
        assert d_out is None
        dXa, dXb, dU, dlam = mahal_bwd(U, lam, X * din, _f64(Xb) * din, dY)
        return dXa * din, dXb * din, dU, dlam
    G = _f64(dY) * dout
    if op in ("apply", "apply_T"):
        dXp, dU = apply_bwd(U, X * din, G, trans=(op == "apply_T"))
        return dXp * din, dU, None
    if op == "sym":
        dXp, dU, dlam = sym_bwd(U, lam, X * din, G)
        return dXp * din, dU, dlam
    raise ValueError(op)


def apply_bwd(U, X, dY, trans: bool = False):
    """Gradients of L = <dY, op(X)> for op = Q (trans=False) or Q^T.

    Returns (dX, dU) with dU the gradient w.r.t. the raw U, shape (h, n)."""
    U, n, h = _shape_U(U)
    X, dY = _f64(X), _f64(dY)
    N = X.shape[0]
    dX = np.empty_like(X)
    dU = np.zeros((h, n))
    _load().orc_apply_bwd(n, h, _p(U), n, int(bool(trans)), _p(X), n, _p(dY), n,
                          N, _p(dX), n, _p(dU), n)
    return dX, dU


def sym_bwd(U, lam, X, dY):
    """Gradients of L = <dY, Q diag(lam) Q^T X>.  Returns (dX, dU, dlam)."""
    U, n, h = _shape_U(U)
    lam, X, dY = _f64(lam), _f64(X), _f64(dY)
    N = X.shape[0]
    dX = np.empty_like(X)
    dU = np.zeros((h, n))
    dlam = np.zeros(n)
    _load().orc_sym_bwd(n, h, _p(U), n, _p(lam), _p(X), n, _p(dY), n, N, _p(dX),
                        n, _p(dU), n, _p(dlam))
    return dX, dU, dlam


def mahal_bwd(U, lam, Xa, Xb, dd):
    """Gradients of L = sum_j dd_j d_j.  Returns (dXa, dXb, dU, dlam)."""
    U, n, h = _shape_U(U)
    lam, Xa, Xb, dd = _f64(lam), _f64(Xa), _f64(Xb), _f64(dd)
    N = Xa.shape[0]
    dXa = np.empty_like(Xa)
    dXb = np.empty_like(Xb)
    dU = np.zeros((h, n))
    dlam = np.zeros(n)
    _load().orc_mahal_bwd(n, h, _p(U), n, _p(lam), _p(Xa), n, _p(Xb), n, _p(dd),
                          N, _p(dXa), _p(dXb), n, _p(dU), n, _p(dlam))
    return dXa, dXb, dU, dlam


def householder_qr(A):
    """Householder QR of a square A (math orientation).

    Returns (V, R): V is (n-1, n) with row k the unit reflector j_k (zeros
    above position k), R upper triangular, and A = J_1 ... J_{n-1} R."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    assert A.shape == (n, n)
    Af = np.ascontiguousarray(A.T)  # column-major buffer
    V = np.zeros((max(n - 1, 0), n))
    R = np.empty((n, n))
    _load().orc_householder_qr(n, _p(Af), n, _p(V), _p(R))
    return V, R.T.copy()
