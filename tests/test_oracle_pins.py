"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with a retyped copy of itself.  Each test uses
an independent fact: hand-derived exact values (tests/golden), invariants of
reflector products (Sec. II-A), the closed form for mutually orthogonal
reflectors (Sec. II-B, eq. in the constrained problem), reproduction of a
random orthonormal matrix from Householder QR reflectors (Result 3, eqs.
ReflectorStructure and theU2), eigen-structure of the symmetric form
(Sec. III-A, eq. thesbar), the Mahalanobis special cases (Sec. IV-C), and
central finite differences for the backward passes.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rng(s):
    return np.random.default_rng(1000 + s)


def random_orthonormal(n, seed):
    """Q factor of a Gaussian matrix (the generator of Sec. II-D / Sec. IV)."""
    A = _rng(seed).standard_normal((n, n))
    Q, _ = np.linalg.qr(A)
    return Q


# --------------------------------------------------------------------------
# hand-derived exact values
# --------------------------------------------------------------------------
def _cases():
    with open(os.path.join(GOLD, "tiny_examples.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_golden_tiny(case):
    U = np.array(case["U"])
    if "Qx" in case:
        x = np.array([case["x"]])
        np.testing.assert_allclose(oracle.apply(U, x)[0], case["Qx"], atol=1e-14)
        np.testing.assert_allclose(oracle.apply(U, x, trans=True)[0], case["QTx"], atol=1e-14)
    if "symx" in case:
        x = np.array([case["x"]])
        np.testing.assert_allclose(oracle.sym(U, case["lam"], x)[0], case["symx"], atol=1e-13)
    if "d" in case:
        d = oracle.mahal(U, case["lam"], np.array([case["xa"]]), np.array([case["xb"]]))
        assert abs(d[0] - case["d"]) < 1e-12
    if "dU" in case:
        dX, dU = oracle.apply_bwd(U, np.array([case["x"]]), np.array([case["g"]]))
        np.testing.assert_allclose(dU, case["dU"], atol=1e-13)
        np.testing.assert_allclose(dX[0], case["dX"], atol=1e-13)


def test_paper_op_counts_and_speedups():
    """The speed-ups quoted at h = ceil(log2 n) are 2n^2 / (4nh) (Sec. IV-C)."""
    with open(os.path.join(GOLD, "op_counts.json")) as f:
        g = json.load(f)
    for c in g["speedups_log2"]["cases"]:
        n = c["n"]
        h = math.ceil(math.log2(n))
        ratio = (2 * n * n) / (4 * n * h)
        assert int(ratio) == c["printed"], (c, ratio)


# --------------------------------------------------------------------------
# invariants of a product of reflectors (Sec. II-A)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,h", [(1, 1), (2, 1), (5, 3), (16, 4), (33, 7), (64, 64)])
def test_dense_Q_orthonormal_and_det(n, h):
    U = _rng(n * 100 + h).standard_normal((h, n))
    Q = oracle.dense_Q(U)
    assert np.abs(Q.T @ Q - np.eye(n)).max() < 1e-13
    assert abs(np.linalg.det(Q) - (-1) ** h) < 1e-10


@pytest.mark.parametrize("n,h", [(7, 3), (40, 6), (100, 7)])
def test_sequential_matches_dense(n, h):
    rng = _rng(n + h)
    U = rng.standard_normal((h, n))
    X = rng.standard_normal((9, n))
    Q = oracle.dense_Q(U)
    assert np.abs(oracle.apply(U, X) - X @ Q.T).max() < 1e-13
    assert np.abs(oracle.apply(U, X, trans=True) - X @ Q).max() < 1e-13


def test_reflector_involution_and_mirror():
    rng = _rng(3)
    n = 12
    for _ in range(5):
        u = rng.standard_normal((1, n))
        X = rng.standard_normal((4, n))
        # H^2 = I
        assert np.abs(oracle.apply(u, oracle.apply(u, X)) - X).max() < 1e-14
        # H uh = -uh, and vectors orthogonal to u are fixed
        uh = u / np.linalg.norm(u)
        assert np.abs(oracle.apply(u, uh) + uh).max() < 1e-15
        w = rng.standard_normal((1, n))
        w -= (w @ uh.T) * uh
        assert np.abs(oracle.apply(u, w) - w).max() < 1e-14


def test_norm_preservation_and_inverse():
    rng = _rng(4)
    n, h = 50, 9
    U = rng.standard_normal((h, n))
    X = rng.standard_normal((20, n))
    Y = oracle.apply(U, X)
    np.testing.assert_allclose(np.linalg.norm(Y, axis=1), np.linalg.norm(X, axis=1), rtol=1e-14)
    assert np.abs(oracle.apply(U, Y, trans=True) - X).max() < 1e-13


def test_orthogonal_complement_fixed():
    """x orthogonal to every u_k  =>  Q x = x."""
    rng = _rng(5)
    n, h = 20, 5
    U = rng.standard_normal((h, n))
    Qb, _ = np.linalg.qr(U.T)  # basis of span(U)
    X = rng.standard_normal((6, n))
    X = X - (X @ Qb) @ Qb.T
    assert np.abs(oracle.apply(U, X) - X).max() < 1e-13


def test_zero_reflector_is_identity():
    rng = _rng(6)
    n = 10
    U = rng.standard_normal((3, n))
    U0 = U.copy()
    U0[1] = 0.0
    X = rng.standard_normal((4, n))
    expect = oracle.apply(U[[0, 2]], X)
    assert np.abs(oracle.apply(U0, X) - expect).max() < 1e-14
    assert abs(np.linalg.det(oracle.dense_Q(U0)) - 1.0) < 1e-12  # two nonzero factors


def test_h_zero_identity():
    X = _rng(7).standard_normal((3, 5))
    assert np.array_equal(oracle.apply(np.zeros((0, 5)), X), X)


# --------------------------------------------------------------------------
# closed form for mutually orthogonal reflectors (Sec. II-B)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,h", [(8, 3), (30, 10), (64, 4)])
def test_orthogonal_set_closed_form(n, h):
    Ut, _ = np.linalg.qr(_rng(n + 7 * h).standard_normal((n, h)))  # orthonormal columns
    closed = np.eye(n) - 2.0 * Ut @ Ut.T
    U = Ut.T
    assert np.abs(oracle.dense_Q(U) - closed).max() < 1e-13
    perm = _rng(1).permutation(h)
    assert np.abs(oracle.dense_Q(U[perm]) - closed).max() < 1e-13  # any order


# --------------------------------------------------------------------------
# Householder QR reproduction (Result 3): J_1 ... J_{n-1} D = U
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 3, 12, 40])
def test_qr_reproduces_orthonormal(n):
    U0 = random_orthonormal(n, n)
    V, R = oracle.householder_qr(U0)
    d = np.sign(np.diag(R))
    # R of an orthonormal matrix is a +-1 diagonal
    assert np.abs(np.abs(np.diag(R)) - 1).max() < 1e-13
    assert np.abs(R - np.diag(np.diag(R))).max() < 1e-13
    Q = oracle.dense_Q(V)
    assert np.abs(Q * d[None, :] - U0).max() < 1e-13
    X = _rng(n).standard_normal((5, n))
    assert np.abs(oracle.apply(V, X) - X @ (U0 * d[None, :]).T).max() < 1e-13
    if n >= 3:
        # the reversed product J_{n-1} ... J_1 is a different matrix
        Qrev = oracle.dense_Q(V[::-1])
        assert np.abs(Qrev * d[None, :] - U0).max() > 1e-2


def test_qr_matches_lapack_up_to_signs():
    A = _rng(11).standard_normal((9, 9))
    V, R = oracle.householder_qr(A)
    _, Rl = np.linalg.qr(A)
    assert np.abs(np.abs(R) - np.abs(Rl)).max() < 1e-12
    assert np.abs(oracle.dense_Q(V) @ R - A).max() < 1e-12
    # leading-zero structure of QR reflectors (remark after Result 3)
    for k in range(V.shape[0]):
        assert np.all(V[k, :k] == 0.0)


@pytest.mark.parametrize("n,h", [(6, 2), (12, 5), (40, 17), (64, 40)])
def test_result3_partial_qr_block_structure(n, h):
    """Result 3 at h < n - 1 (eqs. ReflectorStructure and theU2): the first h
    QR reflectors of an orthonormal U bring it to the block form
    [D_top 0; 0 U~] with D_top a +-1 diagonal and U~ orthonormal, and with
    D = diag(D_top, sign(diag U~)) the error of U ~ J_1 ... J_h D is
    ||U - J_1 ... J_h D||_F^2 = 2(n - h) - 2 sum_i |U~_ii|.  (Eq.
    ReflectorStructure shows I_h in the top block: its reflectors are taken
    with the sign that makes R's diagonal positive; with the textbook sign
    choice v = x + sign(x_1)||x|| e_1 used here the top block carries R's
    signs, which D absorbs.)"""
    U0 = random_orthonormal(n, 100 + n + h)
    V, _ = oracle.householder_qr(U0)
    Vh = V[:h]
    B = oracle.apply(Vh, U0.T, trans=True).T   # column c: J_h ... J_1 U0[:, c]
    top = np.diag(B)[:h]
    assert np.abs(np.abs(top) - 1).max() < 1e-13
    assert np.abs(B[:h, :h] - np.diag(top)).max() < 1e-13
    assert np.abs(B[:h, h:]).max() < 1e-13 and np.abs(B[h:, :h]).max() < 1e-13
    Ut = B[h:, h:]
    assert np.abs(Ut.T @ Ut - np.eye(n - h)).max() < 1e-13
    D = np.concatenate([top, np.sign(np.diag(Ut))])
    err = np.linalg.norm(U0 - oracle.dense_Q(Vh) * D[None, :]) ** 2
    assert abs(err - (2 * (n - h) - 2 * np.abs(np.diag(Ut)).sum())) < 1e-11
    # the reflectors taken in the other order do not give the block form
    if h >= 2:
        Br = oracle.apply(Vh[::-1], U0.T, trans=True).T
        assert np.abs(Br[h:, :h]).max() > 1e-3


def _known_Q(n, seed):
    """Reflectors whose product is a known orthonormal matrix (Result 3)."""
    U0 = random_orthonormal(n, seed)
    V, R = oracle.householder_qr(U0)
    d = np.sign(np.diag(R))
    return V, U0 * d[None, :]


# --------------------------------------------------------------------------
# symmetric form (Sec. III-A)
# --------------------------------------------------------------------------
def test_sym_against_known_eigendecomposition():
    n = 24
    V, Qk = _known_Q(n, 21)
    lam = synth.eig_uniform(n, seed=3)
    X = _rng(21).standard_normal((7, n))
    S = Qk @ np.diag(lam) @ Qk.T
    assert np.abs(oracle.sym(V, lam, X) - X @ S.T).max() < 1e-12


def test_sym_spectrum_and_eigenvectors():
    n, h = 16, 5
    rng = _rng(22)
    U = rng.standard_normal((h, n))
    lam = rng.uniform(-3, 3, n)
    S = oracle.sym(U, lam, np.eye(n)).T  # columns S e_i
    assert np.abs(S - S.T).max() < 1e-13
    np.testing.assert_allclose(np.linalg.eigvalsh(S), np.sort(lam), atol=1e-12)
    Q = oracle.dense_Q(U)
    for i in range(n):
        q = Q[:, i]
        assert np.abs(S @ q - lam[i] * q).max() < 1e-12


def test_sym_constant_spectrum_and_inverse():
    n, h = 30, 6
    rng = _rng(23)
    U = rng.standard_normal((h, n))
    X = rng.standard_normal((5, n))
    assert np.abs(oracle.sym(U, np.full(n, 2.5), X) - 2.5 * X).max() < 1e-13
    lam = rng.uniform(0.5, 2.0, n)
    assert np.abs(oracle.sym(U, 1 / lam, oracle.sym(U, lam, X)) - X).max() < 1e-12


# --------------------------------------------------------------------------
# Mahalanobis distance (Sec. IV-C)
# --------------------------------------------------------------------------
def test_mahal_against_known_metric():
    n = 20
    V, Qk = _known_Q(n, 31)
    lam = synth.eig_uniform(n, seed=4)
    rng = _rng(31)
    Xa, Xb = rng.standard_normal((6, n)), rng.standard_normal((6, n))
    Z = (Xa - Xb) @ Qk  # rows (Q^T v)^T
    expect = (Z * Z) @ lam
    np.testing.assert_allclose(oracle.mahal(V, lam, Xa, Xb), expect, rtol=1e-12)
    S = Qk @ np.diag(lam) @ Qk.T
    quad = np.einsum("ji,ik,jk->j", Xa - Xb, S, Xa - Xb)
    np.testing.assert_allclose(oracle.mahal(V, lam, Xa, Xb), quad, rtol=1e-12)


def test_mahal_special_cases():
    n, h = 15, 4
    rng = _rng(32)
    U = rng.standard_normal((h, n))
    Xa, Xb = rng.standard_normal((8, n)), rng.standard_normal((8, n))
    np.testing.assert_allclose(oracle.mahal(U, np.ones(n), Xa, Xb),
                               ((Xa - Xb) ** 2).sum(1), rtol=1e-13)
    lam = rng.uniform(0.1, 10, n)
    assert np.all(oracle.mahal(U, lam, Xa, Xa) == 0.0)
    np.testing.assert_allclose(oracle.mahal(U, lam, Xa, Xb), oracle.mahal(U, lam, Xb, Xa), rtol=1e-14)


# --------------------------------------------------------------------------
# backward passes: central finite differences and closed forms
# --------------------------------------------------------------------------
def _fd(f, p, eps_rel=1e-6):
    g = np.zeros_like(p)
    it = np.nditer(p, flags=["multi_index"])
    for _ in it:
        idx = it.multi_index
        e = eps_rel * max(1.0, abs(p[idx]))
        pp, pm = p.copy(), p.copy()
        pp[idx] += e
        pm[idx] -= e
        g[idx] = (f(pp) - f(pm)) / (2 * e)
    return g


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("trans", [False, True])
def test_apply_bwd_fd(trans):
    rng = _rng(41 + trans)
    n, h, N = 7, 3, 4
    U = rng.standard_normal((h, n)) * rng.uniform(0.5, 2.0, (h, 1))  # non-unit
    X = rng.standard_normal((N, n))
    G = rng.standard_normal((N, n))
    dX, dU = oracle.apply_bwd(U, X, G, trans)
    fU = _fd(lambda P: np.sum(G * oracle.apply(P, X, trans)), U)
    fX = _fd(lambda P: np.sum(G * oracle.apply(U, P, trans)), X)
    assert _rel(dU, fU) < 1e-6
    assert _rel(dX, fX) < 1e-6
    # closed form: dX = op^T G
    assert np.abs(dX - oracle.apply(U, G, not trans)).max() < 1e-13


def test_sym_bwd_fd():
    rng = _rng(43)
    n, h, N = 6, 3, 3
    U = rng.standard_normal((h, n))
    lam = rng.uniform(0.1, 10, n)
    X = rng.standard_normal((N, n))
    G = rng.standard_normal((N, n))
    dX, dU, dlam = oracle.sym_bwd(U, lam, X, G)
    L = lambda U_, lam_, X_: np.sum(G * oracle.sym(U_, lam_, X_))
    assert _rel(dU, _fd(lambda P: L(P, lam, X), U)) < 1e-6
    assert _rel(dlam, _fd(lambda P: L(U, P, X), lam)) < 1e-6
    assert _rel(dX, _fd(lambda P: L(U, lam, P), X)) < 1e-6
    # closed forms: dX = S G (S symmetric); dlam_i = sum_j (Q^T G)_ij (Q^T X)_ij
    assert np.abs(dX - oracle.sym(U, lam, G)).max() < 1e-12
    PG, PX = oracle.apply(U, G, True), oracle.apply(U, X, True)
    assert np.abs(dlam - (PG * PX).sum(0)).max() < 1e-12


def test_mahal_bwd_fd():
    rng = _rng(44)
    n, h, N = 8, 3, 5
    U = rng.standard_normal((h, n))
    lam = rng.uniform(0.1, 10, n)
    Xa, Xb = rng.standard_normal((N, n)), rng.standard_normal((N, n))
    w = rng.standard_normal(N)
    dXa, dXb, dU, dlam = oracle.mahal_bwd(U, lam, Xa, Xb, w)
    L = lambda U_, lam_, A_, B_: np.dot(w, oracle.mahal(U_, lam_, A_, B_))
    assert _rel(dU, _fd(lambda P: L(P, lam, Xa, Xb), U)) < 1e-6
    assert _rel(dlam, _fd(lambda P: L(U, P, Xa, Xb), lam)) < 1e-6
    assert _rel(dXa, _fd(lambda P: L(U, lam, P, Xb), Xa)) < 1e-6
    assert np.abs(dXa + dXb).max() == 0.0
    Z = oracle.apply(U, Xa - Xb, True)
    assert np.abs(dlam - (w[:, None] * Z * Z).sum(0)).max() < 1e-11


def test_bwd_invariants():
    """Constant spectrum => dU = 0; scale invariance => uh_k^T dU_k = 0;
    zero reflector => zero gradient."""
    rng = _rng(45)
    n, h, N = 12, 4, 6
    U = rng.standard_normal((h, n))
    X, G = rng.standard_normal((N, n)), rng.standard_normal((N, n))
    _, dU, _ = oracle.sym_bwd(U, np.full(n, 3.0), X, G)
    assert np.abs(dU).max() < 1e-12
    Xb = rng.standard_normal((N, n))
    _, _, dU, _ = oracle.mahal_bwd(U, np.full(n, 0.7), X, Xb, rng.standard_normal(N))
    assert np.abs(dU).max() < 1e-12
    _, dU = oracle.apply_bwd(U, X, G)
    assert np.abs((dU * U).sum(1)).max() < 1e-12
    U[2] = 0.0
    _, dU = oracle.apply_bwd(U, X, G)
    assert np.all(dU[2] == 0.0)


# ---------------------------------------------------------------------------
# Diagonal D on either side (eq. 1, Result 3, eq. thesbar)

@pytest.mark.parametrize("n,h", [(12, 5), (40, 17)])
def test_signed_result3_identity_block(n, h):
    """Eq. ReflectorStructure with D in place: D J_h ... J_1 U = [I_h 0; 0 D_1 U~]
    with D_1 U~ of positive diagonal, once D = diag(sign of the top block,
    sign(diag U~)) is put on the output of Q^T = J_h ... J_1 (the transpose of
    Result 3's J_1 ... J_h D); and Result 3's error ||U - J_1 ... J_h D||_F^2 =
    2(n - h) - 2 tr(D_1 U~), with J_1 ... J_h D applied to the identity as Q
    with D on its input."""
    U0 = random_orthonormal(n, 300 + n + h)
    V, _ = oracle.householder_qr(U0)
    Vh = V[:h]
    plain = oracle.apply(Vh, U0.T, trans=True).T
    d = np.concatenate([np.sign(np.diag(plain)[:h]), np.sign(np.diag(plain[h:, h:]))])
    B = oracle.signed("apply_T", Vh, U0.T, d_out=d).T
    assert np.abs(B[:h, :h] - np.eye(h)).max() < 1e-13
    assert np.abs(B[:h, h:]).max() < 1e-13 and np.abs(B[h:, :h]).max() < 1e-13
    assert np.all(np.diag(B[h:, h:]) > 0)
    QD = oracle.signed("apply", Vh, np.eye(n), d_in=d).T   # column j: Q D e_j
    err = np.linalg.norm(U0 - QD) ** 2
    assert abs(err - (2 * (n - h) - 2 * np.trace(B[h:, h:]))) < 1e-11
    # D on the other side of Q^T does not give the identity block
    Bw = oracle.signed("apply_T", Vh, U0.T, d_in=d).T
    assert np.abs(Bw[:h, :h] - np.eye(h)).max() > 1e-3 or np.abs(Bw[h:, :h]).max() > 1e-3


def test_signed_sym_is_symmetric_with_spectrum_lam():
    """Eq. thesbar: D Q diag(lam) Q^T D is symmetric with eigenvalues lam (an
    orthonormal similarity of diag(lam)); with D on one side only it is not
    symmetric.  Its metric gives (x - y)^T S (x - y)."""
    n, h = 24, 6
    rng = _rng(5)
    U = rng.standard_normal((h, n))
    lam = rng.uniform(0.1, 3.0, n)
    d = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    S = oracle.signed("sym", U, np.eye(n), d_in=d, d_out=d, lam=lam)   # row j: S e_j
    assert np.abs(S - S.T).max() < 1e-13
    assert np.abs(np.linalg.eigvalsh(S) - np.sort(lam)).max() < 1e-12
    S1 = oracle.signed("sym", U, np.eye(n), d_out=d, lam=lam)
    assert np.abs(S1 - S1.T).max() > 1e-3
    Xa, Xb = rng.standard_normal((7, n)), rng.standard_normal((7, n))
    dist = oracle.signed("mahal", U, Xa, d_in=d, lam=lam, Xb=Xb)
    ref = np.einsum("ji,ik,jk->j", Xa - Xb, S, Xa - Xb)
    assert np.abs(dist - ref).max() < 1e-12 * np.abs(ref).max()


def test_signed_identity_diagonal_reduces_to_plain_ops():
    """d = 1 everywhere is D = I: the plain ops, bit for bit."""
    n, h, N = 30, 4, 5
    rng = _rng(6)
    U, X, Xb = rng.standard_normal((h, n)), rng.standard_normal((N, n)), rng.standard_normal((N, n))
    lam = rng.uniform(0.1, 2.0, n)
    one = np.ones(n)
    assert np.array_equal(oracle.signed("apply", U, X, d_in=one, d_out=one), oracle.apply(U, X))
    assert np.array_equal(oracle.signed("apply_T", U, X, d_in=one, d_out=one), oracle.apply(U, X, trans=True))
    assert np.array_equal(oracle.signed("sym", U, X, d_in=one, d_out=one, lam=lam), oracle.sym(U, lam, X))
    assert np.array_equal(oracle.signed("mahal", U, X, d_in=one, lam=lam, Xb=Xb), oracle.mahal(U, lam, X, Xb))


@pytest.mark.parametrize("op", ["apply", "apply_T", "sym", "mahal"])
def test_signed_bwd_fd(op):
    """The gradients with diagonals on either side against central differences
    of the forward (eq. 1 / eq. thesbar placements, general diagonals so that a
    dropped or misplaced factor shows)."""
    rng = _rng(60 + len(op))
    n, h, N = 7, 3, 4
    U = rng.standard_normal((h, n)) * rng.uniform(0.5, 2.0, (h, 1))
    X, Xb = rng.standard_normal((N, n)), rng.standard_normal((N, n))
    lam = rng.uniform(0.1, 5.0, n)
    din, dout = rng.uniform(0.5, 2.0, n), rng.uniform(0.5, 2.0, n)
    if op == "mahal":
        w = rng.standard_normal(N)
        dXa, dXb, dU, dlam = oracle.signed_bwd(op, U, X, w, d_in=din, lam=lam, Xb=Xb)
        L = lambda U_, lam_, Xa_, Xb_: np.sum(w * oracle.signed(op, U_, Xa_, d_in=din, lam=lam_, Xb=Xb_))
        assert _rel(dXa, _fd(lambda P: L(U, lam, P, Xb), X)) < 1e-6
        assert _rel(dXb, _fd(lambda P: L(U, lam, X, P), Xb)) < 1e-6
        assert _rel(dU, _fd(lambda P: L(P, lam, X, Xb), U)) < 1e-6
        assert _rel(dlam, _fd(lambda P: L(U, P, X, Xb), lam)) < 1e-6
        return
    G = rng.standard_normal((N, n))
    dX, dU, dlam = oracle.signed_bwd(op, U, X, G, d_in=din, d_out=dout, lam=lam)
    L = lambda U_, lam_, X_: np.sum(G * oracle.signed(op, U_, X_, d_in=din, d_out=dout, lam=lam_))
    assert _rel(dX, _fd(lambda P: L(U, lam, P), X)) < 1e-6
    assert _rel(dU, _fd(lambda P: L(P, lam, X), U)) < 1e-6
    if op == "sym":
        assert _rel(dlam, _fd(lambda P: L(U, P, X), lam)) < 1e-6
    else:
        assert dlam is None
