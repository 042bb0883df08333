"""FP64 oracle of the orthonormal factorisation front-end (Sec. II-B to II-D):
the reflectors that approximate a given orthonormal U.

TEST INFRASTRUCTURE ONLY, like the rest of this package: used by the test
suite, never by the product library.  Library routines serve as steps
(numpy's symmetric and general eigendecompositions, QR); everything else is
written out in the paper's order and notation.

Conventions: U is an (n, n) numpy array in math orientation (U[i, j] is row
i, column j).  Reflector sets are returned as (h, n) arrays, row k the unit
vector of reflector k (or zero: the identity factor, as Result 1 allows),
ordered for the product Q = H_1 H_2 ... H_h of the rest of the oracle and the
library, so that Q approximates U.
"""
from __future__ import annotations

import numpy as np

from . import apply as _apply
from . import householder_qr as _householder_qr


def _sym_eig(U):
    """Z = U + U^T = V diag(z) V^T with z ascending (Sec. II-B)."""
    Z = U + U.T
    z, V = np.linalg.eigh(Z)
    return z, V


def constrained(U, h):
    """Result 1: the best product of h mutually orthogonal reflectors,
    Ubar_1 = I - 2 sum_k u_k u_k^T, takes as u_k the eigenvectors of the
    negative eigenvalues of Z = U + U^T, smallest first (trace minimisation);
    reflectors beyond the n_- negative eigenvalues are zero.  Returns
    (reflectors (h, n), z ascending)."""
    U = np.asarray(U, dtype=np.float64)
    n = U.shape[0]
    z, V = _sym_eig(U)
    R = np.zeros((h, n))
    for k in range(min(h, n)):
        if z[k] < 0:
            R[k] = V[:, k]
    return R, z


def constrained_error(U, h):
    """Eq. expandHouseholderConstrained at the Result 1 choice:
    2n - 2 tr(U) + 2 sum of the h smallest negative z_k; at h = n_- this is
    eq. bestortho, 2n - sum |z_k|."""
    U = np.asarray(U, dtype=np.float64)
    n = U.shape[0]
    z = np.linalg.eigvalsh(U + U.T)
    neg = z[z < 0][:h]
    return 2 * n - 2 * np.trace(U) + 2 * neg.sum()


def unconstrained(U, h, tol=1e-9):
    """Result 2 (Sec. II-C): the full eigendecomposition U = T diag(lam) T^H,
    eigenvalues taken by increasing real part while it is negative:
      Case 1, lam = -1: the real eigenvector is one reflector;
      Case 2, lam = alpha +- i beta: with t_k the eigenvector of the member
        with beta > 0 (unit norm), u_1 = sqrt(2) Re(t_k) and
        u_2 = 2 (gamma Re(t_k) - delta Im(t_k)), gamma = -sqrt(1 + alpha)/2,
        delta = -sqrt(1 - alpha)/2 (eq. theu2): two reflectors.
    The construction builds Ubar_2 = U_m ... U_2 U_1 (each new reflector
    multiplies on the left: ||U - U_2 U_1|| = ||U U_1 - U_2||), so the
    returned rows are in reverse construction order (row 0 = U_m), followed
    by zero rows up to h.  A -1 eigenvalue of multiplicity > 1 has its real
    eigenspace orthonormalised (QR), as the paper's footnote does.  Returns
    (reflectors (h, n), the construction-order list of (case, alpha))."""
    U = np.asarray(U, dtype=np.float64)
    n = U.shape[0]
    lam, T = np.linalg.eig(U)
    steps = []
    # Case 1: eigenvalue -1; its eigenspace from the null space of U + I
    minus = np.where(np.abs(lam + 1.0) < tol)[0]
    if len(minus):
        B = np.real(T[:, minus])
        B, _ = np.linalg.qr(B)
        for j in range(B.shape[1]):
            steps.append((-1.0, 1, B[:, j], None))
    # Case 2: complex pairs with negative real part, the beta > 0 member
    for j in range(n):
        a, b = lam[j].real, lam[j].imag
        if a < 0 and b > tol and abs(lam[j] + 1.0) >= tol:
            t = T[:, j] / np.linalg.norm(T[:, j])
            steps.append((a, 2, t, None))
    steps.sort(key=lambda s: s[0])
    refl, log = [], []
    for a, case, t, _ in steps:
        if len(refl) >= h:
            break
        if case == 1:
            refl.append(t / np.linalg.norm(t))
            log.append((1, -1.0))
            continue
        re, im = np.real(t), np.imag(t)
        refl.append(np.sqrt(2.0) * re)
        log.append((2, a))
        if len(refl) >= h:
            break
        gamma = -np.sqrt(1.0 + a) / 2.0
        delta = -np.sqrt(1.0 - a) / 2.0
        refl.append(2.0 * (gamma * re - delta * im))
        log.append((2, a))
    R = np.zeros((h, n))
    for k, u in enumerate(reversed(refl)):
        R[k] = u
    return R, log


def unconstrained_error_closed(U, h, tol=1e-9):
    """||U - Ubar_2||_F^2 along the Result 2 construction, from the spectrum:
    start at 2n - 2 tr(U) (no reflector); a Case 1 reflector lowers it by 4
    (eigenvalue -2 of Z flipped to +2, eq. flipeigenvalue), the first
    reflector of a Case 2 pair changes it by 4 alpha, the second by -4 (the
    pair's 2 alpha, 2 alpha both become 2).  At h = n_- the total is
    eq. result2, 2 n_+ - sum_{k > n_-} z_k."""
    U = np.asarray(U, dtype=np.float64)
    n = U.shape[0]
    _, log = unconstrained(U, h, tol)
    e = 2 * n - 2 * np.trace(U)
    pair_first = True
    for case, a in log:
        if case == 1:
            e -= 4.0
        elif pair_first:
            e += 4.0 * a
            pair_first = False
        else:
            e -= 4.0
            pair_first = True
    return e


def result2_error(U):
    """Eq. result2 at h = n_-: 2 n_+ - sum of the nonnegative z_k."""
    z = np.linalg.eigvalsh(U + U.T)
    pos = z[z >= 0]
    return 2 * len(pos) - pos.sum()


def qr_partial(U, h):
    """Result 3 (Sec. II-D): the first h reflectors J_1 .. J_h of the
    textbook Householder QR of U and the +-1 diagonal D with
    D J_h ... J_1 U = [D_top 0; 0 D_1 U~] (eq. ReflectorStructure): d_i the
    sign of the i-th diagonal entry of J_h ... J_1 U (sign(0) = +1), which
    makes the top block I_h and D_1 U~ positive on its diagonal.  U is then
    approximated by (J_1 ... J_h) D (eq. theU2).  Returns (reflectors (h, n),
    d (n,))."""
    U = np.asarray(U, dtype=np.float64)
    n = U.shape[0]
    V, _ = _householder_qr(U)
    Vh = V[:h]
    W = _apply(Vh, np.ascontiguousarray(U.T), trans=True).T  # J_h ... J_1 U
    d = np.where(np.diag(W) >= 0, 1.0, -1.0)
    return Vh, d


def result3_bound(n, h):
    """Eq. result1 (Result 3): E ||U - Ubar_2 D||_F^2 <= 2(n - h) - 2 sqrt(2/pi) sqrt(n - h)."""
    return 2.0 * (n - h) - 2.0 * np.sqrt(2.0 / np.pi) * np.sqrt(n - h)
