"""GPU parity of the fused sequential-reflector kernels against the FP64 oracle.

Every case draws seeded inputs once, runs the HIP path through the C ABI and
the oracle on the very same bits (upcast to FP64), and compares output by
output: max over vectors of ||y - y_ref|| / ||y_ref|| for vector outputs,
max relative error for distances, relative Frobenius error for dU and dlam.
Tolerances: FP64 1e-12 (outputs) and 1e-10 (gradients), FP32 1e-5; dU is
also checked reflector by reflector (rel_refl).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import rel_rows, rel_fro, rel_elem, rel_refl

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1811_07624_amd")

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}
GTOL = {torch.float64: 1e-10, torch.float32: 1e-5}


def dev():
    return torch.device("cuda:0")


def make(n, h, N, dtype, seed=0, zero_cols=(), unit=True):
    U = synth.reflectors(n, h, seed=seed, normalize=unit)
    if not unit:
        U = U * synth.host_rng(seed, 99).uniform(0.3, 3.0, (h, 1))
    for k in zero_cols:
        U[k] = 0.0
    X = synth.gaussian((N, n), seed=seed)
    Ut = torch.tensor(U, dtype=dtype, device=dev())
    Xt = torch.tensor(X, dtype=dtype, device=dev())
    return Ut, Xt


def host(t):
    return t.detach().to("cpu", torch.float64).numpy()


SHAPES = [
    # (n, h, N): tiles of 16 and 64 lanes, ragged n and N, chunked reflectors
    (64, 4, 1024), (1, 1, 7), (2, 3, 5), (7, 2, 33), (63, 5, 100), (65, 5, 101),
    (100, 7, 257), (512, 9, 1000), (1000, 10, 129), (1023, 10, 65), (1024, 10, 1000),
    (1025, 3, 17), (2048, 16, 64), (4096, 64, 40), (4096, 3, 9), (513, 6, 31), (700, 12, 3),
    (400, 50, 333),  # FP32: more reflectors than one LDS staging at n <= 512 (8-wave blocks)
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n,h,N", SHAPES)
def test_apply_parity(dtype, n, h, N):
    if dtype == torch.float64 and n > 4096:
        pytest.skip("FP64 fused covers n <= 4096")
    U, X = make(n, h, N, dtype, seed=n + h)
    for trans in (False, True):
        Y = P.apply_raw(U, X, trans=trans)
        torch.cuda.synchronize()
        ref = oracle.apply(host(U), host(X), trans=trans)
        assert rel_rows(host(Y), ref) < TOL[dtype], (trans, rel_rows(host(Y), ref))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n,h,N", SHAPES)
def test_sym_parity(dtype, n, h, N):
    U, X = make(n, h, N, dtype, seed=2 * n + h)
    lam = torch.tensor(synth.eig_uniform(n, seed=n), dtype=dtype, device=dev())
    Y = P.sym_raw(U, lam, X)
    torch.cuda.synchronize()
    ref = oracle.sym(host(U), host(lam), host(X))
    assert rel_rows(host(Y), ref) < TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n,h,N", SHAPES)
def test_mahal_parity(dtype, n, h, N):
    U, Xa = make(n, h, N, dtype, seed=3 * n + h)
    Xb = torch.tensor(synth.gaussian((N, n), seed=5, stream=synth.STREAM_XB), dtype=dtype,
                      device=dev())
    lam = torch.tensor(synth.eig_uniform(n, seed=n), dtype=dtype, device=dev())
    d = P.mahal_raw(U, lam, Xa, Xb)
    torch.cuda.synchronize()
    ref = oracle.mahal(host(U), host(lam), host(Xa), host(Xb))
    assert rel_elem(host(d), ref) < TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_edge_cases(dtype):
    n = 37
    # h = 0: identity, copy, scaling, plain squared distance
    U0 = torch.zeros((0, n), dtype=dtype, device=dev())
    X = torch.randn((11, n), dtype=dtype, device=dev())
    assert torch.equal(P.apply_raw(U0, X), X)
    lam = torch.rand(n, dtype=dtype, device=dev()) + 0.5
    torch.testing.assert_close(P.sym_raw(U0, lam, X), X * lam, rtol=0, atol=0)
    # zero reflector columns are identities
    U, X = make(n, 5, 13, dtype, zero_cols=(1, 3))
    ref = oracle.apply(host(U), host(X))
    assert rel_rows(host(P.apply_raw(U, X)), ref) < TOL[dtype]
    # non-unit reflector vectors are normalised
    U, X = make(n, 4, 9, dtype, unit=False)
    assert rel_rows(host(P.apply_raw(U, X)), oracle.apply(host(U), host(X))) < TOL[dtype]
    # N = 0
    E = torch.empty((0, n), dtype=dtype, device=dev())
    assert P.apply_raw(U, E).shape == (0, n)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_strided_and_in_place(dtype):
    n, h, N = 129, 6, 50
    U, X = make(n, h, N, dtype)
    big = torch.randn((N, n + 3), dtype=dtype, device=dev())
    big[:, :n] = X
    Xv = big[:, :n]  # leading dimension n + 3: scalar-access path
    Y = P.apply_raw(U, Xv)
    ref = oracle.apply(host(U), host(X))
    assert rel_rows(host(Y), ref) < TOL[dtype]
    Xi = X.clone()
    P.apply_raw(U, Xi, out=Xi)  # in place
    assert rel_rows(host(Xi), ref) < TOL[dtype]


def test_qx_n64_h4_fp64_full():
    """n=64, h=4, N=1024 FP64, both Q X and Q^T X: relative error <= 1e-12."""
    U, X = make(64, 4, 1024, torch.float64, seed=0)
    for trans in (False, True):
        Y = P.apply_raw(U, X, trans=trans)
        ref = oracle.apply(host(U), host(X), trans=trans)
        assert rel_rows(host(Y), ref) < 1e-12


# ----------------------------------------------------------------------------
# backward
# ----------------------------------------------------------------------------
# the last two have more reflector data than the on-chip budget (read through
# the caches instead of staged in LDS)
BSHAPES = [(64, 4, 300), (7, 3, 5), (100, 7, 129), (512, 9, 1000), (1024, 10, 77),
           (300, 20, 50), (2048, 5, 20), (33, 0, 10), (16, 40, 9), (1024, 40, 30), (2048, 24, 12)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n,h,N", BSHAPES)
def test_apply_bwd_parity(dtype, n, h, N):
    U, X = make(n, h, N, dtype, seed=7 * n + h, unit=False)
    G = torch.tensor(synth.gaussian((N, n), seed=1, stream=synth.STREAM_G), dtype=dtype,
                     device=dev())
    for trans in (False, True):
        dX, dU = P.apply_bwd_raw(U, X, G, trans=trans)
        torch.cuda.synchronize()
        rdX, rdU = oracle.apply_bwd(host(U), host(X), host(G), trans=trans)
        assert rel_rows(host(dX), rdX) < TOL[dtype]
        if h:
            assert rel_fro(host(dU), rdU) < GTOL[dtype], rel_fro(host(dU), rdU)
            assert rel_refl(host(dU), rdU) < GTOL[dtype], rel_refl(host(dU), rdU)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n,h,N", BSHAPES)
def test_sym_bwd_parity(dtype, n, h, N):
    U, X = make(n, h, N, dtype, seed=11 * n + h)
    lam = torch.tensor(synth.eig_uniform(n, seed=n), dtype=dtype, device=dev())
    G = torch.tensor(synth.gaussian((N, n), seed=2, stream=synth.STREAM_G), dtype=dtype,
                     device=dev())
    dX, dU, dlam = P.sym_bwd_raw(U, lam, X, G)
    torch.cuda.synchronize()
    rdX, rdU, rdlam = oracle.sym_bwd(host(U), host(lam), host(X), host(G))
    assert rel_rows(host(dX), rdX) < TOL[dtype]
    assert rel_fro(host(dlam), rdlam) < GTOL[dtype]
    if h:
        assert rel_fro(host(dU), rdU) < GTOL[dtype]
        assert rel_refl(host(dU), rdU) < GTOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n,h,N", BSHAPES)
def test_mahal_bwd_parity(dtype, n, h, N):
    U, Xa = make(n, h, N, dtype, seed=13 * n + h)
    Xb = torch.tensor(synth.gaussian((N, n), seed=3, stream=synth.STREAM_XB), dtype=dtype,
                      device=dev())
    lam = torch.tensor(synth.eig_uniform(n, seed=n), dtype=dtype, device=dev())
    w = torch.tensor(synth.gaussian((N,), seed=4, stream=synth.STREAM_W), dtype=dtype,
                     device=dev())
    dXa, dXb, dU, dlam = P.mahal_bwd_raw(U, lam, Xa, Xb, w)
    torch.cuda.synchronize()
    rXa, rXb, rU, rlam = oracle.mahal_bwd(host(U), host(lam), host(Xa), host(Xb), host(w))
    assert rel_rows(host(dXa), rXa) < TOL[dtype]
    assert torch.equal(dXb, -dXa)
    assert rel_fro(host(dlam), rlam) < GTOL[dtype]
    if h:
        assert rel_fro(host(dU), rU) < GTOL[dtype]
        assert rel_refl(host(dU), rU) < GTOL[dtype]


@pytest.mark.parametrize("op", ["apply", "apply_T", "sym", "mahal"])
def test_fused_bwd_fp32_n4096_h64(op):
    """FP32 gradients at the headline shape (n = 4096, h = 64: 1 MiB of
    reflectors, read through the caches) against the oracle, to the FP32
    tolerances of the other backward tests."""
    n, h, N, dtype = 4096, 64, 6, torch.float32
    U, X = make(n, h, N, dtype, seed=5, unit=False)
    G = torch.tensor(synth.gaussian((N, n), seed=6, stream=synth.STREAM_G), dtype=dtype, device=dev())
    lam = torch.tensor(synth.eig_uniform(n, seed=7), dtype=dtype, device=dev())
    if op in ("apply", "apply_T"):
        dX, dU = P.apply_bwd_raw(U, X, G, trans=op == "apply_T")
        torch.cuda.synchronize()
        rdX, rdU = oracle.apply_bwd(host(U), host(X), host(G), trans=op == "apply_T")
    elif op == "sym":
        dX, dU, dlam = P.sym_bwd_raw(U, lam, X, G)
        torch.cuda.synchronize()
        rdX, rdU, rdlam = oracle.sym_bwd(host(U), host(lam), host(X), host(G))
        assert rel_fro(host(dlam), rdlam) < GTOL[dtype]
    else:
        w = torch.tensor(synth.gaussian((N,), seed=8, stream=synth.STREAM_W), dtype=dtype, device=dev())
        dX, _, dU, dlam = P.mahal_bwd_raw(U, lam, X, G, w)
        torch.cuda.synchronize()
        rdX, _, rdU, rdlam = oracle.mahal_bwd(host(U), host(lam), host(X), host(G), host(w))
        assert rel_fro(host(dlam), rdlam) < GTOL[dtype]
    assert rel_rows(host(dX), rdX) < TOL[dtype]
    assert rel_fro(host(dU), rdU) < GTOL[dtype], rel_fro(host(dU), rdU)
    assert rel_refl(host(dU), rdU) < GTOL[dtype], rel_refl(host(dU), rdU)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n,h,N", [(512, 9, 1000), (100, 7, 129), (1024, 40, 30), (33, 0, 10),
                                   (7, 3, 5), (64, 4, 0),
                                   (400, 90, 77)])  # FP32: 8-wave staging plan, record in two chunks
def test_mahal_bwd_from_record(dtype, n, h, N):
    """Distances with the record of dot products (hh_mahalanobis_save) equal the
    plain ones exactly, and the backward from the record meets the oracle to the
    stated tolerances; it differs from the plain backward only by the rounding
    of the dot products (the forward's reduction order)."""
    U, Xa = make(n, h, N, dtype, seed=17 * n + h)
    Xb = torch.tensor(synth.gaussian((N, n), seed=3, stream=synth.STREAM_XB), dtype=dtype, device=dev())
    lam = torch.tensor(synth.eig_uniform(n, seed=n), dtype=dtype, device=dev())
    w = torch.tensor(synth.gaussian((N,), seed=4, stream=synth.STREAM_W), dtype=dtype, device=dev())
    d0 = P.mahal_raw(U, lam, Xa, Xb)
    d1, rec = P.mahal_raw(U, lam, Xa, Xb, save=True)
    g0 = P.mahal_bwd_raw(U, lam, Xa, Xb, w)
    g1 = P.mahal_bwd_raw(U, lam, Xa, Xb, w, saved=rec)
    torch.cuda.synchronize()
    assert torch.equal(d0, d1)
    if N == 0:
        return
    rXa, rXb, rU, rlam = oracle.mahal_bwd(host(U), host(lam), host(Xa), host(Xb), host(w))
    dXa, dXb, dU, dlam = g1
    assert rel_rows(host(dXa), rXa) < TOL[dtype]
    assert torch.equal(dXb, -dXa)
    assert rel_fro(host(dlam), rlam) < GTOL[dtype]
    if h:
        assert rel_fro(host(dU), rU) < GTOL[dtype]
        assert rel_refl(host(dU), rU) < GTOL[dtype]
        # the record holds the forward's dot products u_k^T s_{k-1}, pair j in row j
        es = 8 if dtype == torch.float64 else 4
        hp = -(-h * es // 16) * 16 // es  # rows padded to 16 bytes
        rows = rec[: hp * N * es].view(dtype).view(N, hp)
        assert not rows[:, h:].any()
        dots = rows[:, :h].T
        ref = oracle_dots(host(U), host(Xa) - host(Xb))
        assert np.abs(host(dots) - ref).max() <= TOL[dtype] * np.abs(ref).max()
    for a, b in zip(g0, g1):
        assert rel_fro(host(a), host(b)) < GTOL[dtype]


def oracle_dots(U, V):
    """u_k^T s_{k-1} along the chain s_k = H_k s_{k-1} that Q^T v applies
    (unit u_k = U_k / ||U_k||), one row per reflector, by the definition."""
    h = U.shape[0]
    S = V.T.copy()
    out = np.zeros((h, V.shape[0]))
    for k in range(h):
        u = U[k] / np.linalg.norm(U[k])
        out[k] = u @ S
        S -= 2.0 * np.outer(u, out[k])
    return out


def test_bwd_n_zero_writes_zero_grads():
    U, _ = make(40, 3, 1, torch.float32)
    E = torch.empty((0, 40), dtype=torch.float32, device=dev())
    lam = torch.ones(40, dtype=torch.float32, device=dev())
    dX, dU, dlam = P.sym_bwd_raw(U, lam, E, E)
    torch.cuda.synchronize()
    assert torch.count_nonzero(dU) == 0 and torch.count_nonzero(dlam) == 0


def test_bwd_deterministic():
    U, X = make(512, 9, 5000, torch.float32)
    G = torch.randn_like(X)
    a = P.apply_bwd_raw(U, X, G)[1]
    b = P.apply_bwd_raw(U, X, G)[1]
    assert torch.equal(a, b)


def test_fd_fp64_gpu():
    """Central finite differences of the GPU FP64 forward against the GPU
    backward at tiny shapes (n <= 16, h <= 4, N <= 64)."""
    n, h, N = 12, 3, 16
    U, X = make(n, h, N, torch.float64, seed=5, unit=False)
    lam = torch.tensor(synth.eig_uniform(n, seed=1), dtype=torch.float64, device=dev())
    G = torch.randn_like(X)

    def loss(Up, lamp):
        return float((G * P.sym_raw(Up, lamp, X)).sum())

    _, dU, dlam = P.sym_bwd_raw(U, lam, X, G)
    fdU = torch.zeros_like(U)
    for k in range(h):
        for i in range(n):
            e = 1e-6 * max(1.0, abs(float(U[k, i])))
            Up, Um = U.clone(), U.clone()
            Up[k, i] += e
            Um[k, i] -= e
            fdU[k, i] = (loss(Up, lam) - loss(Um, lam)) / (2 * e)
    assert rel_fro(host(dU), host(fdU)) < 1e-6
    fdl = torch.zeros_like(lam)
    for i in range(n):
        lp, lm = lam.clone(), lam.clone()
        lp[i] += 1e-6
        lm[i] -= 1e-6
        fdl[i] = (loss(U, lp) - loss(U, lm)) / 2e-6
    assert rel_fro(host(dlam), host(fdl)) < 1e-6


def test_autograd_functions():
    n, h, N = 64, 4, 32
    U, X = make(n, h, N, torch.float64)
    U.requires_grad_(True)
    X.requires_grad_(True)
    lam = torch.tensor(synth.eig_uniform(n), dtype=torch.float64, device=dev(), requires_grad=True)
    Xb = torch.randn_like(X)
    w = torch.randn(N, dtype=torch.float64, device=dev())
    L = (P.mahalanobis(U, lam, X, Xb) * w).sum() + P.sym_apply(U, lam, X).square().sum() \
        + P.apply(U, X).sum() + P.apply_T(U, X).sum()
    L.backward()
    # reference gradients from the oracle
    Uh, Xh, lh, Xbh, wh = host(U), host(X), host(lam), host(Xb), host(w)
    _, _, gU1, gl1 = oracle.mahal_bwd(Uh, lh, Xh, Xbh, wh)
    gX1, _, _, _ = oracle.mahal_bwd(Uh, lh, Xh, Xbh, wh)
    Ys = oracle.sym(Uh, lh, Xh)
    gX2, gU2, gl2 = oracle.sym_bwd(Uh, lh, Xh, 2 * Ys)
    gX3, gU3 = oracle.apply_bwd(Uh, Xh, np.ones_like(Xh), False)
    gX4, gU4 = oracle.apply_bwd(Uh, Xh, np.ones_like(Xh), True)
    assert rel_fro(host(U.grad), gU1 + gU2 + gU3 + gU4) < 1e-10
    assert rel_fro(host(lam.grad), gl1 + gl2) < 1e-10
    assert rel_fro(host(X.grad), gX1 + gX2 + gX3 + gX4) < 1e-10


@pytest.mark.parametrize("n,h", [(4096, 64), (1024, 10), (64, 4)])
def test_fused_orthogonality(n, h):
    """E = Q^T Q - I of the fused FP32 path (applied to the identity, E formed
    in FP64): max |E_ij| within the FP32 tolerance, for Q and Q^T."""
    U = torch.tensor(synth.reflectors(n, h, seed=0), dtype=torch.float32, device=dev())
    I = torch.eye(n, dtype=torch.float32, device=dev())
    for trans in (False, True):
        Qt = P.apply_raw(U, I, trans=trans).double()
        E = Qt @ Qt.T - torch.eye(n, dtype=torch.float64, device=dev())
        assert float(E.abs().max()) < TOL[torch.float32], trans
