"""Pins of the SHF / SHF-SU oracle (oracle/shf.py, Sec. III-B, Algorithm 1)
against what the paper and the mathematics fix, on the CPU.

* Eq. objectivefunctionS3: ||A - U_k B U_k||_F^2 = ||A||^2 + ||B||^2
  - 2 tr(AB) + 4 C(u) for unit u (a dropped factor in C fails it); the
  gradient of eq. gradient against central differences; the arcs of eqs.
  combine and iterate stay on the unit sphere.
* Descent: after the initialisation every iteration lowers the error or keeps
  it (Sec. III-B: the search contains the previous point), for SHF and
  SHF-SU; SHF-SU ends no worse than SHF.
* Closed forms: with h = 0, SHF-SU's spectrum update leaves exactly the
  off-diagonal part of D S D; a matrix that is exactly U_1 diag(sbar) U_1 with
  one reflector is recovered (error ~ 0) by SHF-SU with h = 1.
* Result 4: on random S = (X + X^T)/2 the mean SHF-SU error lies below the
  mean of eq. result4's bound.
"""
import numpy as np
import pytest

from oracle import shf as H


def rand_sym(n, seed):
    X = np.random.default_rng(seed).standard_normal((n, n))
    return (X + X.T) / 2


def test_objective_identity_and_gradient():
    rng = np.random.default_rng(0)
    n = 9
    A, B = rand_sym(n, 1), rand_sym(n, 2)
    for _ in range(5):
        u = rng.standard_normal(n)
        u /= np.linalg.norm(u)
        R = H.refl(u)
        lhs = np.linalg.norm(A - R @ B @ R) ** 2
        rhs = (np.linalg.norm(A) ** 2 + np.linalg.norm(B) ** 2 - 2 * np.trace(A @ B)
               + 4 * H.C(u, A, B))
        assert abs(lhs - rhs) < 1e-10 * lhs
        g = H.grad_C(u, A, B)
        fd = np.zeros(n)
        for i in range(n):
            e = np.zeros(n)
            e[i] = 1e-6
            fd[i] = (H.C(u + e, A, B) - H.C(u - e, A, B)) / 2e-6
        assert np.abs(g - fd).max() < 1e-6 * np.abs(g).max()
    p = rng.standard_normal(n)
    p /= np.linalg.norm(p)
    q = rng.standard_normal(n)
    q -= (q @ p) * p
    q /= np.linalg.norm(q)
    for gm in np.linspace(0, np.sqrt(2), 7):
        for sg in (1.0, -1.0):
            assert abs(np.linalg.norm(H.sphere_point(p, q, gm, sg)) - 1) < 1e-14


@pytest.mark.parametrize("n,h,seed", [(12, 2, 0), (20, 3, 1), (24, 5, 2)])
def test_descent_and_spectrum_update(n, h, seed):
    S = rand_sym(n, seed)
    _, _, _, e = H.shf(S, h, 8)
    _, _, _, e2 = H.shf(S, h, 8, spectrum_update=True)
    assert all(b <= a + 1e-9 * a for a, b in zip(e[:-1], e[1:]))
    assert all(b <= a + 1e-9 * a for a, b in zip(e2[:-1], e2[1:]))
    assert e2[-1] <= e[-1] + 1e-9 * e[-1]
    # the reported error is the dense ||S - Sbar||^2 of the returned factors
    U, sb, d, e3 = H.shf(S, h, 3, spectrum_update=True)
    assert abs(np.linalg.norm(S - H.approx(sb, d, U)) ** 2 - e3[-1]) < 1e-9 * e3[-1]


def test_no_reflectors_closed_form():
    S = rand_sym(15, 3)
    U, sb, d, e = H.shf(S, 0, 3, spectrum_update=True)
    DSD = d[:, None] * S * d[None, :]
    assert np.allclose(sb, np.diag(DSD))
    off = DSD - np.diag(np.diag(DSD))
    assert abs(e[-1] - np.linalg.norm(off) ** 2) < 1e-10 * e[-1]


@pytest.mark.parametrize("seed", range(4))
def test_exact_one_reflector_recovered(seed):
    n = 24
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(n)
    u /= np.linalg.norm(u)
    s = rng.standard_normal(n)
    s = s[np.argsort(-np.abs(s))]
    R = H.refl(u)
    S = R @ np.diag(s) @ R
    _, _, _, e = H.shf(S, 1, 30, spectrum_update=True)
    assert e[-1] < 1e-10 * np.linalg.norm(S) ** 2


def test_result4_expected_error():
    n, h = 24, 6
    es, bs = [], []
    for seed in range(6):
        S = rand_sym(n, 100 + seed)
        es.append(H.shf(S, h, 30, spectrum_update=True)[3][-1])
        bs.append(H.result4_bound(S, h))
    assert np.mean(es) <= np.mean(bs)
