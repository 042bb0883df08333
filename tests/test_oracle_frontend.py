"""Pins of the front-end oracle (oracle/frontend.py) against what Sec. II-B to
II-D and the mathematics fix, on the CPU.

* Result 1: the dense product's error equals eq. expandHouseholderConstrained
  at every h and eq. bestortho (2n - sum |z_k|) at h = n_-; no other set of
  h orthonormal reflectors (random samples) does better (trace minimisation).
* Result 2: the dense product's error follows the per-step closed form of the
  construction (Case 1: -4; Case 2: +4 alpha, then -4) at every h, equals
  eq. result2 (2 n_+ - sum z_k) at h = n_-, never exceeds Result 1's, and the
  second reflector of a Case 2 pair is an eigenvector of U U_1 with eigenvalue
  -1 (the step the paper's choice of gamma and delta is made for).
* Hadamard and Fourier (Sec. IV-A): H + H^T has half its eigenvalues at -2,
  half at +2, so n/2 reflectors reproduce H exactly and Results 1 and 2 give
  the same errors; F + F^H has floor((n+2)/4) eigenvalues at -2 and
  floor((n+4)/4) at +2.
* Result 3: the partial-QR reflectors with D give the block form of
  eq. ReflectorStructure, and the mean error over random orthonormal U
  matches eq. result1's expectation (the bound is attained by QR).
"""
import numpy as np
import pytest

import oracle
from oracle import frontend as F


def rand_orth(n, seed):
    U, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, n)))
    return U


def dense(R, n):
    return oracle.dense_Q(R) if R.shape[0] else np.eye(n)


def sylvester_hadamard(n):
    H = np.ones((1, 1))
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    return H / np.sqrt(n)


@pytest.mark.parametrize("n,seed", [(8, 0), (9, 1), (40, 2), (63, 3)])
def test_result1_closed_form_and_optimality(n, seed):
    U = rand_orth(n, seed)
    z = np.linalg.eigvalsh(U + U.T)
    nneg = int((z < 0).sum())
    for h in range(0, nneg + 2):
        R, _ = F.constrained(U, h)
        G = R @ R.T
        nz = np.linalg.norm(R, axis=1) > 0
        assert np.allclose(G[np.ix_(nz, nz)], np.eye(int(nz.sum())), atol=1e-12)  # orthonormal
        e = np.linalg.norm(U - dense(R, n)) ** 2
        assert abs(e - F.constrained_error(U, h)) < 1e-10 * (1 + e)
    R, _ = F.constrained(U, nneg)
    assert abs(np.linalg.norm(U - dense(R, n)) ** 2 - (2 * n - np.abs(z).sum())) < 1e-10 * n
    # any other h orthonormal reflectors do no better
    h = max(1, nneg // 2)
    best = F.constrained_error(U, h)
    rng = np.random.default_rng(seed + 100)
    for _ in range(20):
        W, _ = np.linalg.qr(rng.standard_normal((n, h)))
        Q = np.eye(n) - 2 * W @ W.T
        assert np.linalg.norm(U - Q) ** 2 >= best - 1e-10


@pytest.mark.parametrize("n,seed", [(8, 0), (9, 1), (40, 2), (63, 3), (16, 7)])
def test_result2_closed_form(n, seed):
    U = rand_orth(n, seed)
    z = np.linalg.eigvalsh(U + U.T)
    nneg = int((z < 0).sum())
    prev = np.inf
    for h in range(0, nneg + 2):
        R, _ = F.unconstrained(U, h)
        assert np.allclose(np.linalg.norm(R[np.linalg.norm(R, axis=1) > 0], axis=1), 1.0)
        e = np.linalg.norm(U - dense(R, n)) ** 2
        assert abs(e - F.unconstrained_error_closed(U, h)) < 1e-9 * (1 + e)
        assert e <= F.constrained_error(U, h) + 1e-9
        assert e <= prev + 1e-9  # each reflector lowers the error or keeps it
        prev = e
    R, _ = F.unconstrained(U, nneg)
    assert abs(np.linalg.norm(U - dense(R, n)) ** 2 - F.result2_error(U)) < 1e-9 * n


def test_result2_second_reflector_is_minus_one_eigenvector():
    """Sec. II-C, Case 2: with u_1 = sqrt(2) Re(t_k), the u_2 of eq. theu2
    satisfies U U_1 u_2 = -u_2; a wrong sign of gamma, delta or beta fails."""
    for seed in range(5):
        U = rand_orth(12, seed + 20)
        R, log = F.unconstrained(U, 40)
        k = [i for i, (case, _) in enumerate(log) if case == 2][0]  # first Case 2 pair
        m = len(log)
        u1, u2 = R[m - 1 - k], R[m - 2 - k]  # rows are in reverse construction order
        U1 = np.eye(12) - 2 * np.outer(u1, u1)
        assert np.allclose(U @ U1 @ u2, -u2, atol=1e-10)


@pytest.mark.parametrize("n", [4, 16, 64])
def test_hadamard_exact_with_half_the_reflectors(n):
    H = sylvester_hadamard(n)
    z = np.linalg.eigvalsh(H + H.T)
    assert (np.abs(z + 2) < 1e-12).sum() == n // 2 and (np.abs(z - 2) < 1e-12).sum() == n // 2
    for h in (1, n // 4, n // 2):
        e1 = np.linalg.norm(H - dense(F.constrained(H, h)[0], n)) ** 2
        e2 = np.linalg.norm(H - dense(F.unconstrained(H, h)[0], n)) ** 2
        assert abs(e1 - e2) < 1e-9 and abs(e1 - (2 * n - 4 * h)) < 1e-9
    assert np.linalg.norm(H - dense(F.constrained(H, n // 2)[0], n)) < 1e-12


@pytest.mark.parametrize("n", range(8, 18))
def test_fourier_eigenvalue_counts(n):
    Fm = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n) / np.sqrt(n)
    z = np.linalg.eigvalsh(Fm + Fm.conj().T)
    assert (np.abs(z + 2) < 1e-9).sum() == (n + 2) // 4
    assert (np.abs(z - 2) < 1e-9).sum() == (n + 4) // 4
    assert (np.abs(z) < 1e-9).sum() == n - (n + 2) // 4 - (n + 4) // 4


@pytest.mark.parametrize("n,h", [(20, 5), (33, 32)])
def test_result3_block_form(n, h):
    U = rand_orth(n, n + h)
    V, d = F.qr_partial(U, h)
    W = d[:, None] * oracle.apply(V, np.ascontiguousarray(U.T), trans=True).T  # D J_h..J_1 U
    assert np.allclose(W[:h, :h], np.eye(h), atol=1e-12)
    assert np.abs(W[:h, h:]).max() < 1e-12 and np.abs(W[h:, :h]).max() < 1e-12
    assert (np.diag(W)[h:] >= 0).all()
    e = np.linalg.norm(U - dense(V, n) * d) ** 2
    assert abs(e - (2 * (n - h) - 2 * np.trace(W[h:, h:]))) < 1e-10 * n


@pytest.mark.parametrize("n,h", [(64, 8), (64, 32), (128, 16)])
def test_result3_expected_error(n, h):
    errs = []
    for s in range(40):
        U = rand_orth(n, s)
        V, d = F.qr_partial(U, h)
        errs.append(np.linalg.norm(U - dense(V, n) * d) ** 2)
    mean, se = np.mean(errs), np.std(errs) / np.sqrt(len(errs))
    assert abs(mean - F.result3_bound(n, h)) < 4 * se + 1e-3 * n
