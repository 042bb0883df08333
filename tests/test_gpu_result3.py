"""The GPU path on the paper's Result 3 construction (eqs. ReflectorStructure
and theU2): the first h < n - 1 Householder QR reflectors J_1 .. J_h of a random
orthonormal U (formed by the oracle's textbook QR), applied as Q^T = J_h ... J_1
to the columns of U, give the block form [D_top 0; 0 U~] with D_top a +-1
diagonal.  QR reflectors have leading zeros (the remark after Result 3); the
kernels treat them as dense vectors.  Fused FP64/FP32 and compact-WY BF16/FP16;
tolerances 1e-12 (FP64), 1e-5 (FP32), 2e-2 (16-bit) on the block entries.
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1811_07624_amd")


def qr_case(n, h, seed):
    A = np.random.default_rng(seed).standard_normal((n, n))
    U0, _ = np.linalg.qr(A)
    V, _ = oracle.householder_qr(U0)
    return U0, V[:h]


CASES = [("f64", 40, 17, 1e-12), ("f32", 256, 100, 1e-5), ("bf16", 256, 100, 2e-2),
         ("f16", 64, 24, 2e-2), ("bf16", 1024, 128, 2e-2)]
DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}


@pytest.mark.parametrize("dname,n,h,tol", CASES)
def test_result3_block_structure(dname, n, h, tol):
    dt = DT[dname]
    U0, Vh = qr_case(n, h, seed=n + h)
    param = torch.float64 if dt == torch.float64 else torch.float32
    Ud = torch.tensor(Vh, dtype=param, device="cuda")
    # rows of the batch are the columns of U0
    X = torch.tensor(np.ascontiguousarray(U0.T), dtype=torch.float64, device="cuda").to(dt)
    B = P.apply_raw(Ud, X, trans=True, compute=dt).double().cpu().numpy().T
    top = np.diag(B)[:h]
    assert np.abs(np.abs(top) - 1).max() < tol
    assert np.abs(B[:h, :h] - np.diag(top)).max() < tol
    assert np.abs(B[:h, h:]).max() < tol
    assert np.abs(B[h:, :h]).max() < tol
    Ut = B[h:, h:]
    assert np.abs(Ut.T @ Ut - np.eye(n - h)).max() < 4 * tol
    # and the oracle, given the same rounded input, agrees vector by vector
    ref = oracle.apply(Vh.astype(np.float32).astype(np.float64) if param == torch.float32 else Vh,
                       X.double().cpu().numpy(), trans=True).T
    assert np.abs(B - ref).max() < tol
