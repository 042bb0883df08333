"""GPU parity of the orthonormal factorisation front-end (Sec. II-B to II-D)
against the FP64 oracle (oracle/frontend.py), through the C ABI.

What is unique is compared directly: the spectrum of U + U^T; Result 1's
operator I - 2 sum u_k u_k^T (the span of the chosen eigenvectors); Result 2's
product of whole Case 1 / Case 2 steps (a pair's two reflections compose a
rotation of its invariant plane that does not depend on the phase of the
eigenvector); the QR reflectors and signs (the sign convention fixes them).
Where several answers are correct (h cutting a pair) the closed-form error is
compared.  The reflectors then run through the transform kernels: the
approximation errors ||U - Q||_F^2 of the GPU path match the closed forms
(eqs. bestortho, result2, and 2(n - h) - 2 tr(D_1 U~) for Result 3).
Tolerance: 1e-10 relative on errors and operators (FP64 Jacobi with 1e-15
off-diagonal convergence).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import frontend as F

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1811_07624_amd")


def dev():
    return torch.device("cuda:0")


def rand_orth(n, seed):
    U, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, n)))
    return U


def gpu(U, h, method):
    R, d, z = P.factor_orthonormal(torch.tensor(U, device=dev()), h, method)
    torch.cuda.synchronize()
    return R.cpu().numpy(), d.cpu().numpy(), None if z is None else z.cpu().numpy()


def q_gpu(R, n, d=None):
    """The dense operator Q diag(d) applied by the transform kernels (FP64):
    row j of the result is (Q D e_j)^T."""
    Ut = torch.tensor(R, device=dev())
    E = torch.eye(n, dtype=torch.float64, device=dev())
    if d is None:
        Y = P.apply_raw(Ut, E)
    else:
        Y = P.signed_raw("apply", Ut, E, d_in=torch.tensor(d, device=dev()))
    return Y.cpu().numpy().T


def dense(R, n):
    return oracle.dense_Q(R) if R.shape[0] else np.eye(n)


SIZES = [(8, 0), (9, 1), (64, 2), (101, 3), (256, 4)]


@pytest.mark.parametrize("n,seed", SIZES)
def test_constrained(n, seed):
    U = rand_orth(n, seed)
    zr = np.linalg.eigvalsh(U + U.T)
    nneg = int((zr < 0).sum())
    for h in sorted({1, nneg // 2, nneg, nneg + 3}):
        R, d, z = gpu(U, h, "constrained")
        assert np.abs(z - zr).max() < 1e-12 * n
        assert (d == 1).all()
        Rr, _ = F.constrained(U, h)
        Q = q_gpu(R, n)
        # the eigenvalues of U + U^T come in equal pairs (complex pairs of U):
        # the operator is unique unless h splits an eigenvalue's eigenspace
        if h >= nneg or zr[h] - zr[h - 1] > 1e-6:
            assert np.abs(Q - dense(Rr, n)).max() < 1e-10
        e = np.linalg.norm(U - Q) ** 2
        assert abs(e - F.constrained_error(U, h)) < 1e-10 * (1 + e)
        if h >= nneg:
            assert abs(e - (2 * n - np.abs(zr).sum())) < 1e-10 * n


@pytest.mark.parametrize("n,seed", SIZES)
def test_unconstrained(n, seed):
    U = rand_orth(n, seed)
    zr = np.linalg.eigvalsh(U + U.T)
    nneg = int((zr < 0).sum())
    for h in sorted({1, 2, 3, nneg // 2, nneg - 1, nneg}):
        if h < 1:
            continue
        R, d, z = gpu(U, h, "unconstrained")
        Q = q_gpu(R, n)
        e = np.linalg.norm(U - Q) ** 2
        assert abs(e - F.unconstrained_error_closed(U, h)) < 1e-9 * (1 + e), h
        Rr, log = F.unconstrained(U, h)
        # whole steps only (no Case 2 pair cut in half): the operator is unique
        if sum(1 for case, _ in log if case == 2) % 2 == 0:
            assert np.abs(Q - dense(Rr, n)).max() < 1e-9, h
    R, _, _ = gpu(U, nneg, "unconstrained")
    e = np.linalg.norm(U - q_gpu(R, n)) ** 2
    assert abs(e - F.result2_error(U)) < 1e-9 * n


@pytest.mark.parametrize("n", [16, 64])
def test_hadamard(n):
    """H + H^T = 2H has only the eigenvalues -2 and 2, n/2 times each: n/2
    reflectors reproduce H (Sec. IV-A).  Such a multiple spectrum converges
    linearly in the cyclic Jacobi method (random U converge quadratically,
    about 9 sweeps), so after the 16 sweeps the eigenspaces are accurate to
    about 1e-10: tolerance 1e-9 here."""
    H = np.ones((1, 1))
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    H = H / np.sqrt(n)
    for method in ("constrained", "unconstrained"):
        R, _, z = gpu(H, n // 2, method)
        assert (np.abs(z + 2) < 1e-12).sum() == n // 2
        assert np.abs(q_gpu(R, n) - H).max() < 1e-9


@pytest.mark.parametrize("n,h", [(50, 10), (64, 63), (200, 120), (513, 40)])
def test_qr(n, h):
    U = rand_orth(n, n + h)
    R, d, z = gpu(U, h, "qr")
    assert z is None
    Rr, dr = F.qr_partial(U, h)
    assert np.abs(R - Rr).max() < 1e-12
    assert (d == dr).all()
    for k in range(h):  # the leading zeros of the remark after Result 3
        assert (R[k, :k] == 0).all()
    Q = q_gpu(R, n, d)
    W = dr[:, None] * oracle.apply(Rr, np.ascontiguousarray(U.T), trans=True).T
    e = np.linalg.norm(U - Q) ** 2
    assert abs(e - (2 * (n - h) - 2 * np.trace(W[h:, h:]))) < 1e-10 * n
    if h == n - 1:
        assert np.abs(Q - U).max() < 1e-12


def test_h_zero_and_tiny():
    U = rand_orth(5, 9)
    R, d, z = gpu(U, 0, "unconstrained")
    assert R.shape == (0, 5) and np.allclose(np.sort(z), np.linalg.eigvalsh(U + U.T))
    R, d, z = gpu(np.array([[-1.0]]), 3, "unconstrained")  # n = 1: one Case 1 reflector
    assert np.allclose(np.abs(R[0]), [1.0]) and np.allclose(R[1:], 0.0)
