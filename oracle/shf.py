"""FP64 oracle of the Symmetric Householder Factorisation (Sec. III-B,
Algorithm 1, SHF and SHF-SU): S ~ Sbar = D U_1 ... U_h diag(sbar) U_h ... U_1 D
(eq. thesbar).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy in the
paper's order and notation; numpy's eigh serves as the eigensolver step.

Readings where the paper leaves a choice open (each also stated in DESIGN):
  * the one-dimensional searches over gamma in [0, sqrt 2] (Matlab's fminbnd
    in the paper) are a 65-point grid followed by 40 golden-section steps on
    the two grid intervals around the best point; gamma = 0 is on the grid,
    so a step never increases C;
  * u_dagger-dagger from the Kronecker eigenvector: V = a b^T for the chosen
    eigenvectors a (of A_k) and b (of B_k); the best symmetric rank-one
    approximation of V + V^T is along a + b or a - b (v is defined up to
    sign), the one with the larger (u^T A u)(u^T B u) is taken;
  * the diagonal D (eq. optimaldiagonal) minimises ||S - D B_0 D||_F^2 one
    entry at a time in index order, flipping d_i when that lowers the error
    (the printed inequality would pick the sign that raises it);
  * "until convergence" of the inner descent: at most 20 steps, stopping when
    a step lowers C by no more than 1e-12 max(1, |C|); the outer loop stops
    early when the relative progress of the error is below 1e-8 (the "10e-8"
    of the text, read as 1e-8).
"""
from __future__ import annotations

import numpy as np

GRID = 65
GOLDEN = 40
INNER = 20
INNER_TOL = 1e-12
OUTER_TOL = 1e-8


def refl(u):
    """U_k = I - 2 u u^T (u unit or zero)."""
    return np.eye(len(u)) - 2.0 * np.outer(u, u)


def C(u, A, B, M=None):
    """Eq. theRk: C(u) = u^T (A B + B A) u - 2 (u^T A u)(u^T B u); M = AB + BA
    may be passed in."""
    if M is None:
        M = A @ B + B @ A
    return u @ M @ u - 2.0 * (u @ A @ u) * (u @ B @ u)


def grad_C(u, A, B, M=None):
    """Eq. gradient."""
    if M is None:
        M = A @ B + B @ A
    return 2.0 * M @ u - 4.0 * ((u @ A @ u) * B + (u @ B @ u) * A) @ u


def sphere_point(p, q, gamma, sign):
    """(1 - gamma^2/2) p + sign sqrt(gamma^2 - gamma^4/4) q: unit when p, q are
    orthonormal (eqs. combine and iterate)."""
    return (1.0 - gamma * gamma / 2.0) * p + sign * np.sqrt(max(gamma * gamma - gamma ** 4 / 4.0, 0.0)) * q


def line_search(f):
    """Minimise f over gamma in [0, sqrt 2]: grid, then golden section."""
    g = np.linspace(0.0, np.sqrt(2.0), GRID)
    vals = np.array([f(x) for x in g])
    i = int(np.argmin(vals))
    lo, hi = g[max(i - 1, 0)], g[min(i + 1, GRID - 1)]
    best_x, best_v = g[i], vals[i]
    r = (np.sqrt(5.0) - 1.0) / 2.0
    x1, x2 = hi - r * (hi - lo), lo + r * (hi - lo)
    f1, f2 = f(x1), f(x2)
    for _ in range(GOLDEN):
        if f1 <= f2:
            hi, x2, f2 = x2, x1, f1
            x1 = hi - r * (hi - lo)
            f1 = f(x1)
        else:
            lo, x1, f1 = x1, x2, f2
            x2 = lo + r * (hi - lo)
            f2 = f(x2)
    for x, v in ((x1, f1), (x2, f2)):
        if v < best_v:
            best_x, best_v = x, v
    return best_x, best_v


def build_A(S, d, U, k):
    """Eq. ak: A_k = U_{k-1} ... U_1 D S D U_1 ... U_{k-1} (k 0-based: the
    reflectors before k)."""
    A = (d[:, None] * S) * d[None, :]
    for j in range(k):
        R = refl(U[j])
        A = R @ A @ R
    return A


def build_B(sbar, U, k):
    """Eq. bk: B_k = U_{k+1} ... U_h diag(sbar) U_h ... U_{k+1}."""
    B = np.diag(sbar)
    for j in range(len(U) - 1, k, -1):
        R = refl(U[j])
        B = R @ B @ R
    return B


def approx(sbar, d, U):
    """Sbar = D U_1 ... U_h diag(sbar) U_h ... U_1 D (eq. thesbar)."""
    B0 = build_B(sbar, U, -1)
    return (d[:, None] * B0) * d[None, :]


def init_reflector(A, B):
    """Eq. combine: u_dagger (smallest eigenvalue of AB + BA), u_ddagger
    (Kronecker step), orthogonalised (eq. processtheinitial), then the best
    point of the arc between them."""
    M = A @ B + B @ A
    _, Vm = np.linalg.eigh(M)
    ud = Vm[:, 0]
    la, Va = np.linalg.eigh(A)
    lb, Vb = np.linalg.eigh(B)
    cand = [(la[0] * lb[0], Va[:, 0], Vb[:, 0]), (la[0] * lb[-1], Va[:, 0], Vb[:, -1]),
            (la[-1] * lb[0], Va[:, -1], Vb[:, 0]), (la[-1] * lb[-1], Va[:, -1], Vb[:, -1])]
    _, a, b = max(cand, key=lambda c: c[0])
    best, best_q = None, -np.inf
    for v in (a + b, a - b):
        nv = np.linalg.norm(v)
        if nv < 1e-12:
            continue
        v = v / nv
        q = (v @ A @ v) * (v @ B @ v)
        if q > best_q:
            best, best_q = v, q
    udd = best - (ud @ best) * ud
    nu = np.linalg.norm(udd)
    if nu < 1e-12:
        return ud
    udd = udd / nu
    best_u, best_c = ud, C(ud, A, B, M)
    for sign in (1.0, -1.0):
        gm, cv = line_search(lambda x: C(sphere_point(ud, udd, x, sign), A, B, M))
        if cv < best_c:
            best_u, best_c = sphere_point(ud, udd, gm, sign), cv
    return best_u


def descend(u, A, B):
    """Eqs. gradient and iterate: projected, normalised gradient; the step
    along the great circle that minimises C; until a step gains nothing."""
    M = A @ B + B @ A
    c = C(u, A, B, M)
    for _ in range(INNER):
        g = grad_C(u, A, B, M)
        g = g - (u @ g) * u
        ng = np.linalg.norm(g)
        if ng < 1e-14:
            break
        g = g / ng
        gm, cv = line_search(lambda x: C(sphere_point(u, g, x, -1.0), A, B, M))
        if c - cv <= INNER_TOL * max(1.0, abs(c)):
            if cv < c:
                u, c = sphere_point(u, g, gm, -1.0), cv
            break
        u, c = sphere_point(u, g, gm, -1.0), cv
    return u


def update_D(S, sbar, U, d):
    """Eq. optimaldiagonal read as the minimiser of ||S - D B_0 D||_F^2, one
    entry at a time: flip d_i when the off-diagonal part of row i matches
    better with the other sign."""
    B0 = build_B(sbar, U, -1)
    d = d.copy()
    n = len(d)
    for i in range(n):
        mask = np.arange(n) != i
        bi = d[i] * d[mask] * B0[i, mask]
        si = S[i, mask]
        if np.linalg.norm(si + bi) < np.linalg.norm(si - bi):
            d[i] = -d[i]
    return d


def error(S, sbar, d, U):
    return float(np.linalg.norm(S - approx(sbar, d, U)) ** 2)


def shf(S, h, K, spectrum_update=False):
    """Algorithm 1 (SHF; SHF-SU with spectrum_update): returns
    (reflectors (h, n), sbar, d, errors) with errors[0] after the
    initialisation and errors[i] after iteration i (||S - Sbar||_F^2)."""
    S = np.asarray(S, dtype=np.float64)
    n = S.shape[0]
    s = np.linalg.eigvalsh(S)
    sbar = s[np.argsort(-np.abs(s), kind="stable")]
    U = np.zeros((h, n))
    d = np.ones(n)
    for k in range(h):
        U[k] = init_reflector(build_A(S, d, U, k), build_B(sbar, U, k))
    d = update_D(S, sbar, U, d)
    if spectrum_update:
        sbar = np.diag(build_A(S, d, U, h)).copy()
    errs = [error(S, sbar, d, U)]
    for _ in range(K):
        for k in range(h):
            U[k] = descend(U[k], build_A(S, d, U, k), build_B(sbar, U, k))
        d = update_D(S, sbar, U, d)
        if spectrum_update:  # eq. updateofsbar: sbar = diag(Ubar^T S Ubar)
            sbar = np.diag(build_A(S, d, U, h)).copy()
        errs.append(error(S, sbar, d, U))
        if errs[-2] - errs[-1] < OUTER_TOL * errs[-2]:
            break
    return U, sbar, d, errs


def result4_bound(S, h):
    """Eq. result4 for one S: sum_{i > h} sigma_i^2 - (n - h)/2."""
    sig = np.sort(np.abs(np.linalg.eigvalsh(S)))[::-1]
    return float((sig[h:] ** 2).sum() - (len(sig) - h) / 2.0)
