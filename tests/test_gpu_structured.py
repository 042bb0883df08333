"""Reflectors with the sparsity of Householder QR (the remark after Result 3:
j_k = [0_{k-1}; j~_k], at most n - k + 1 nonzeros, 4(n - k + 1) operations per
application): the fused kernels skip the leading zero chunks of each
reflector.  The skipped terms are exact zeros, so the results must meet the
same tolerances as dense reflectors (FP64 1e-12, FP32 1e-5 against the FP64
oracle), including h = n - 1, where Result 3's construction reproduces U
exactly (J_1 ... J_{n-1} D = U).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import rel_elem, rel_rows

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1811_07624_amd")

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def dev():
    return torch.device("cuda:0")


def host(t):
    return t.detach().to("cpu", torch.float64).numpy()


# (n, h, N): chunk sizes of 16-lane rows (64 FP32 / 32 FP64 rows per chunk)
# and 64-lane rows, ragged n, h = n - 1, h < n - 1, LDS chunks of reflectors
SHAPES = [(512, 511, 300), (300, 299, 65), (64, 63, 129), (1024, 1023, 40), (2048, 300, 20),
          (100, 40, 33), (4096, 200, 9)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n,h,N", SHAPES)
def test_structured_parity(dtype, n, h, N):
    U = torch.tensor(synth.structured_reflectors(n, h, seed=n + h), dtype=dtype, device=dev())
    X = torch.tensor(synth.gaussian((N, n), seed=n), dtype=dtype, device=dev())
    lam = torch.tensor(synth.eig_uniform(n, seed=n), dtype=dtype, device=dev())
    Xb = torch.tensor(synth.gaussian((N, n), seed=n, stream=synth.STREAM_XB), dtype=dtype,
                      device=dev())
    Uh, Xh = host(U), host(X)
    for trans in (False, True):
        Y = P.apply_raw(U, X, trans=trans, algo="fused_qr")
        Yd = P.apply_raw(U, X, trans=trans, algo="fused")
        torch.cuda.synchronize()
        assert rel_rows(host(Y), oracle.apply(Uh, Xh, trans=trans)) < TOL[dtype], trans
        assert torch.equal(Y, Yd), trans  # the skipped terms are exact zeros
    Y = P.sym_raw(U, lam, X, algo="fused_qr")
    d = P.mahal_raw(U, lam, X, Xb, algo="fused_qr")
    torch.cuda.synchronize()
    assert rel_rows(host(Y), oracle.sym(Uh, host(lam), Xh)) < TOL[dtype]
    assert rel_elem(host(d), oracle.mahal(Uh, host(lam), Xh, host(Xb))) < TOL[dtype]
    assert torch.equal(Y, P.sym_raw(U, lam, X, algo="fused"))
    assert torch.equal(d, P.mahal_raw(U, lam, X, Xb, algo="fused"))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_skip_kernels_on_dense_reflectors(dtype):
    """The skipping kernels on reflectors without leading zeros (and with a
    zero reflector and ragged LDS chunks) give the dense kernels' results."""
    n, h, N = 700, 150, 77
    U = torch.tensor(synth.reflectors(n, h, seed=3), dtype=dtype, device=dev())
    U[5] = 0
    X = torch.tensor(synth.gaussian((N, n), seed=3), dtype=dtype, device=dev())
    for trans in (False, True):
        assert torch.equal(P.apply_raw(U, X, trans=trans, algo="fused_qr"),
                           P.apply_raw(U, X, trans=trans, algo="fused"))


@pytest.mark.parametrize("dtype,n", [(torch.float64, 200), (torch.float32, 512), (torch.float64, 1024)])
def test_result3_full_reproduction(dtype, n):
    """h = n - 1 QR reflectors of a random orthonormal U0 with the sign
    diagonal D (Result 3, eq. theU2 and eq. ReflectorStructure): Q D e_j, run
    on the GPU with D on the input, reproduces the columns of U0."""
    rng = np.random.default_rng(n)
    U0, _ = np.linalg.qr(rng.standard_normal((n, n)))
    V, R = oracle.householder_qr(U0)
    Dd = np.sign(np.diag(R))
    U = torch.tensor(V[: n - 1], dtype=dtype, device=dev())
    d = torch.tensor(Dd, dtype=dtype, device=dev())
    E = torch.eye(n, dtype=dtype, device=dev())
    cols = P.signed_raw("apply", U, E, d_in=d, algo="fused_qr").double().cpu().numpy()  # (Q D e_j)^T
    assert rel_rows(cols, U0.T) < TOL[dtype]
