"""Householder-reflector transforms on AMD Instinct MI355X (gfx950).

Applies Q = H_1 ... H_h (H_k = I - 2 uh_k uh_k^T), its transpose, the symmetric
form Q diag(lam) Q^T and the Mahalanobis distance of the learned metric to
batches of vectors, with gradients, through the C ABI of libhh.so.
"""
from .transforms import (apply, apply_T, sym_apply, mahalanobis, signed, apply_raw, sym_raw, mahal_raw,
                         signed_raw, signed_bwd_raw, forward_noalloc_raw, factor_orthonormal, shf, knn, knn_raw, apply_bwd_raw, sym_bwd_raw, mahal_bwd_raw)
from ._lib import lib, HHError, LIB_PATH

__all__ = ["apply", "apply_T", "sym_apply", "mahalanobis", "signed", "apply_raw", "sym_raw", "mahal_raw",
           "signed_raw", "signed_bwd_raw", "forward_noalloc_raw", "factor_orthonormal", "shf", "knn", "knn_raw", "apply_bwd_raw", "sym_bwd_raw", "mahal_bwd_raw", "lib", "HHError", "LIB_PATH"]
