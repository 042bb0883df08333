"""GPU parity of the compact-WY matrix-core path (BF16 / FP16) against the FP64
oracle.

The oracle receives exactly the bits handed to the GPU: the data rounded to the
16-bit type (round to nearest even) and the FP32 reflector vectors, upcast to
FP64.  Rounding the normalised reflectors to 16 bits inside the library is
part of the path's error.  Tolerance: max over vectors of
||y - y_ref|| / ||y_ref|| <= 2e-2 for both 16-bit types.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import rel_rows, rel_refl

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1811_07624_amd")

TOL16 = 2e-2
DT = {"bf16": torch.bfloat16, "f16": torch.float16}


def dev():
    return torch.device("cuda:0")


def host(t):
    return t.detach().to("cpu", torch.float64).numpy()


def make(n, h, N, dt, seed=0):
    U = torch.tensor(synth.reflectors(n, h, seed=seed), dtype=torch.float32, device=dev())
    X = torch.tensor(synth.gaussian((N, n), seed=seed), dtype=torch.float32, device=dev()).to(dt)
    return U, X


# n * hp >= 2^19 selects the streaming kernel (tiles of 128 vectors, ragged
# tails included); smaller shapes the register-resident one.
SHAPES = [(4096, 64, 1000), (256, 10, 33), (512, 9, 100), (1024, 64, 50), (2048, 100, 40),
          (8192, 128, 20), (4096, 1, 17), (1000, 7, 31), (64, 3, 5), (8192, 64, 300),
          (4096, 100, 129), (6144, 128, 257), (64, 100, 9), (32, 64, 40),  # these two: h > n
          (6144, 50, 77),  # resident kernel with 1024-row wave slices
          (2000, 65, 37), (8184, 33, 21)]  # h padded 65 -> 128; n short of the largest padding


@pytest.mark.parametrize("dname", ["bf16", "f16"])
@pytest.mark.parametrize("n,h,N", SHAPES)
def test_wy_apply_parity(dname, n, h, N):
    dt = DT[dname]
    U, X = make(n, h, N, dt, seed=n + h)
    for trans in (False, True):
        Y = P.apply_raw(U, X, trans=trans, compute=dt)
        torch.cuda.synchronize()
        assert Y.dtype == dt
        ref = oracle.apply(host(U), host(X), trans=trans)
        err = rel_rows(host(Y), ref)
        assert err < TOL16, (trans, err)


@pytest.mark.parametrize("dname", ["bf16", "f16"])
@pytest.mark.parametrize("n,h,N", [(512, 9, 64), (1024, 64, 40), (2048, 100, 16), (4096, 128, 133),
                                   (8192, 64, 70), (6144, 50, 77), (4096, 64, 45)])
def test_wy_sym_parity(dname, n, h, N):
    dt = DT[dname]
    U, X = make(n, h, N, dt, seed=3 * n + h)
    lam = torch.tensor(synth.eig_loguniform(n, seed=1), dtype=torch.float32, device=dev())
    Y = P.sym_raw(U, lam, X, compute=dt)
    torch.cuda.synchronize()
    ref = oracle.sym(host(U), host(lam), host(X))
    assert rel_rows(host(Y), ref) < TOL16


def test_wy_edge_cases():
    dt = torch.bfloat16
    n = 128
    # h = 0: identity (zero reflectors are padded in)
    U0 = torch.zeros((0, n), dtype=torch.float32, device=dev())
    X = torch.randn((9, n), device=dev()).to(dt)
    assert torch.equal(P.apply_raw(U0, X, compute=dt), X)
    # zero reflector columns are identities
    U, X = make(n, 5, 21, dt)
    U[2] = 0
    ref = oracle.apply(host(U), host(X))
    assert rel_rows(host(P.apply_raw(U, X, compute=dt)), ref) < TOL16
    # N = 0
    E = torch.empty((0, n), dtype=dt, device=dev())
    assert P.apply_raw(U, E, compute=dt).shape == (0, n)
    # ragged tile: N not a multiple of the 32-vector tile
    U, X = make(n, 5, 45, dt)
    ref = oracle.apply(host(U), host(X))
    assert rel_rows(host(P.apply_raw(U, X, compute=dt)), ref) < TOL16


@pytest.mark.parametrize("n,h,N", [(256, 12, 40), (8192, 64, 37)])  # resident / streaming kernel
def test_wy_ld_and_in_place(n, h, N):
    dt = torch.bfloat16
    U, X = make(n, h, N, dt)
    big = torch.zeros((N, n + 16), dtype=dt, device=dev())
    big[:, :n] = X
    Y = P.apply_raw(U, big[:, :n], compute=dt)
    ref = oracle.apply(host(U), host(X))
    assert rel_rows(host(Y), ref) < TOL16
    assert torch.count_nonzero(big[:, n:]) == 0
    Xi = X.clone()
    P.apply_raw(U, Xi, compute=dt, out=Xi)
    assert rel_rows(host(Xi), ref) < TOL16


# Unit roundoff of the 16-bit types (8 and 11 significant bits).
UNIT = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}


@pytest.mark.parametrize("dname,n,h", [("bf16", 4096, 64), ("f16", 8192, 128),
                                       ("bf16", 1024, 64), ("f16", 1024, 64)])
def test_wy_orthogonality(dname, n, h):
    """Apply the path to the identity (exact in 16 bits) and measure
    E = Q^T Q - I in FP64, at the benchmark shapes (n = 4096, h = 64 BF16;
    n = 8192, h = 128 FP16) for Q and Q^T.

    T is formed from the rounded reflectors, so the blocked operator is
    orthogonal up to FP32 accumulation; what remains is the rounding of each
    output entry to the 16-bit type, q^ = q (1 + e).  Then
    E_ij ~ q_i^T d_j + d_i^T q_j with ||d_j|| <= u, so max |E_ij| <= 2u + u^2,
    and ||E||_F^2 ~ 2 sum_j ||d_j||^2 = 2 n rho^2 with rho the rms relative
    rounding error, 2^(1-p) / sqrt(12) * sqrt(3 / (8 ln 2)) = 0.425 u for
    log-uniform mantissas: ||E||_F / sqrt(n) ~ 0.60 u.  Bounds: 2.1 u and
    0.75 u."""
    dt = DT[dname]
    u = UNIT[dname]
    U = torch.tensor(synth.reflectors(n, h, seed=0), dtype=torch.float32, device=dev())
    I = torch.eye(n, device=dev()).to(dt)
    for trans in (False, True):
        Qt = P.apply_raw(U, I, trans=trans, compute=dt).double()  # rows: columns of Q
        E = Qt @ Qt.T - torch.eye(n, dtype=torch.float64, device=dev())
        mx, fro = float(E.abs().max()), float(E.norm() / np.sqrt(n))
        del Qt, E
        assert mx < 2.1 * u, (trans, mx)
        assert fro < 0.75 * u, (trans, fro)


def test_wy_matches_fused_fp32():
    n, h, N = 4096, 64, 256
    U, Xf = make(n, h, N, torch.float32, seed=2)
    Xb = Xf.to(torch.bfloat16)
    Yw = P.apply_raw(U, Xb, compute=torch.bfloat16).float()
    Yf = P.apply_raw(U, Xb.float())
    assert rel_rows(host(Yw), host(Yf)) < TOL16


# ----------------------------------------------------------------------------
# backward of the WY path
# ----------------------------------------------------------------------------
from tests._util import rel_fro  # noqa: E402

BSHAPES = [(512, 9, 100), (1024, 64, 50), (4096, 64, 300), (2048, 100, 40), (8192, 128, 64),
           (256, 3, 1000), (64, 1, 7), (8192, 64, 131), (6144, 50, 77)]


@pytest.mark.parametrize("dname", ["bf16", "f16"])
@pytest.mark.parametrize("n,h,N", BSHAPES)
def test_wy_apply_bwd_parity(dname, n, h, N):
    dt = DT[dname]
    U, X = make(n, h, N, dt, seed=5 * n + h)
    Uraw = U * torch.linspace(0.5, 2.0, h, device=dev())[:, None]  # non-unit columns
    G = torch.tensor(synth.gaussian((N, n), seed=2, stream=synth.STREAM_G), dtype=torch.float32,
                     device=dev()).to(dt)
    for trans in (False, True):
        dX, dU = P.apply_bwd_raw(Uraw, X, G, trans=trans, compute=dt)
        torch.cuda.synchronize()
        rdX, rdU = oracle.apply_bwd(host(Uraw), host(X), host(G), trans=trans)
        assert rel_rows(host(dX), rdX) < TOL16, (trans, rel_rows(host(dX), rdX))
        assert rel_fro(host(dU), rdU) < TOL16, (trans, rel_fro(host(dU), rdU))
        assert rel_refl(host(dU), rdU) < TOL16, rel_refl(host(dU), rdU)


@pytest.mark.parametrize("dname", ["bf16", "f16"])
@pytest.mark.parametrize("n,h,N", [(512, 9, 100), (1024, 64, 40), (2048, 100, 33), (8192, 128, 48)])
def test_wy_sym_bwd_parity(dname, n, h, N):
    dt = DT[dname]
    U, X = make(n, h, N, dt, seed=7 * n + h)
    lam = torch.tensor(synth.eig_loguniform(n, seed=2), dtype=torch.float32, device=dev())
    G = torch.tensor(synth.gaussian((N, n), seed=3, stream=synth.STREAM_G), dtype=torch.float32,
                     device=dev()).to(dt)
    dX, dU, dlam = P.sym_bwd_raw(U, lam, X, G, compute=dt)
    torch.cuda.synchronize()
    rdX, rdU, rdlam = oracle.sym_bwd(host(U), host(lam), host(X), host(G))
    assert rel_rows(host(dX), rdX) < TOL16, rel_rows(host(dX), rdX)
    assert rel_fro(host(dU), rdU) < TOL16, rel_fro(host(dU), rdU)
    assert rel_refl(host(dU), rdU) < TOL16, rel_refl(host(dU), rdU)
    assert rel_fro(host(dlam), rdlam) < TOL16, rel_fro(host(dlam), rdlam)


def test_wy_bwd_edge_cases():
    dt = torch.bfloat16
    n = 256
    U, X = make(n, 6, 0, dt)
    E = torch.empty((0, n), dtype=dt, device=dev())
    lam = torch.ones(n, device=dev())
    dX, dU, dlam = P.sym_bwd_raw(U, lam, E, E, compute=dt)
    torch.cuda.synchronize()
    assert torch.count_nonzero(dU) == 0 and torch.count_nonzero(dlam) == 0
    # h = 0: dX = S G = lam * G; dlam = sum_j G X
    U0 = torch.zeros((0, n), device=dev())
    _, X = make(n, 1, 40, dt)
    G = torch.randn((40, n), device=dev()).to(dt)
    lam = torch.rand(n, device=dev()) + 0.5
    dX, dU, dlam = P.sym_bwd_raw(U0, lam, X, G, compute=dt)
    rdX, _, rdlam = oracle.sym_bwd(np.zeros((0, n)), host(lam), host(X), host(G))
    assert rel_rows(host(dX), rdX) < TOL16
    assert rel_fro(host(dlam), rdlam) < 1e-3
    # zero reflector column: zero gradient column
    U, X = make(n, 5, 33, dt)
    U[1] = 0
    G = torch.randn((33, n), device=dev()).to(dt)
    _, dU = P.apply_bwd_raw(U, X, G, compute=dt)
    assert torch.count_nonzero(dU[1]) == 0
    _, rdU = oracle.apply_bwd(host(U), host(X), host(G))
    assert rel_fro(host(dU), rdU) < TOL16
    assert rel_refl(host(dU), rdU) < TOL16, rel_refl(host(dU), rdU)


def test_wy_stream_sym_ld_in_place():
    """Streaming kernel (n * hp >= 2^19): leading dimensions larger than n,
    in-place symmetric form, and the backward reading strided inputs."""
    dt = torch.float16
    n, h, N = 4096, 120, 50
    U, X = make(n, h, N, dt, seed=11)
    lam = torch.tensor(synth.eig_loguniform(n, seed=4), dtype=torch.float32, device=dev())
    big = torch.zeros((N, n + 40), dtype=dt, device=dev())
    big[:, :n] = X
    ref = oracle.sym(host(U), host(lam), host(X))
    Y = P.sym_raw(U, lam, big[:, :n], compute=dt)
    assert rel_rows(host(Y), ref) < TOL16
    P.sym_raw(U, lam, big[:, :n], compute=dt, out=big[:, :n])
    assert rel_rows(host(big[:, :n]), ref) < TOL16
    assert torch.count_nonzero(big[:, n:]) == 0
    Gb = torch.zeros((N, n + 8), dtype=dt, device=dev())
    G = torch.tensor(synth.gaussian((N, n), seed=5, stream=synth.STREAM_G), dtype=torch.float32,
                     device=dev()).to(dt)
    Gb[:, :n] = G
    Xb = torch.zeros((N, n + 16), dtype=dt, device=dev())
    Xb[:, :n] = X
    dX, dU, dlam = P.sym_bwd_raw(U, lam, Xb[:, :n], Gb[:, :n], compute=dt)
    rdX, rdU, rdlam = oracle.sym_bwd(host(U), host(lam), host(X), host(G))
    assert rel_rows(host(dX), rdX) < TOL16
    assert rel_fro(host(dU), rdU) < TOL16
    assert rel_refl(host(dU), rdU) < TOL16, rel_refl(host(dU), rdU)
    assert rel_fro(host(dlam), rdlam) < TOL16


def test_wy_bwd_deterministic():
    dt = torch.float16
    U, X = make(1024, 64, 500, dt)
    G = torch.randn_like(X)
    a = P.apply_bwd_raw(U, X, G, compute=dt)[1]
    b = P.apply_bwd_raw(U, X, G, compute=dt)[1]
    assert torch.equal(a, b)


def test_wy_autograd():
    dt = torch.bfloat16
    n, h, N = 512, 16, 64
    U, X = make(n, h, N, dt)
    U.requires_grad_(True)
    lam = torch.tensor(synth.eig_uniform(n), dtype=torch.float32, device=dev(), requires_grad=True)
    G = torch.randn((N, n), device=dev()).to(dt)
    Y = P.sym_apply(U, lam, X, compute=dt)
    (Y.float() * G.float()).sum().backward()
    _, rdU, rdlam = oracle.sym_bwd(host(U), host(lam), host(X), host(G))
    assert rel_fro(host(U.grad), rdU) < TOL16
    assert rel_refl(host(U.grad), rdU) < TOL16, rel_refl(host(U.grad), rdU)
    assert rel_fro(host(lam.grad), rdlam) < TOL16


# ----------------------------------------------------------------------------
# coefficient record of the forward, taken by the backward
# ----------------------------------------------------------------------------
# resident kernel (n * hp < 2^19) and streaming kernel, ragged N
SAVED_SHAPES = [(512, 9, 100), (4096, 64, 300), (8192, 128, 48), (2048, 100, 33), (64, 1, 7)]


@pytest.mark.parametrize("dname", ["bf16", "f16"])
@pytest.mark.parametrize("n,h,N", SAVED_SHAPES)
@pytest.mark.parametrize("kind", ["apply", "apply_T", "sym"])
def test_wy_saved_record(dname, n, h, N, kind):
    dt = DT[dname]
    U, X = make(n, h, N, dt, seed=11 * n + h)
    Uraw = U * torch.linspace(0.5, 2.0, h, device=dev())[:, None]
    lam = torch.tensor(synth.eig_loguniform(n, seed=3), dtype=torch.float32, device=dev())
    G = torch.tensor(synth.gaussian((N, n), seed=4, stream=synth.STREAM_G), dtype=torch.float32,
                     device=dev()).to(dt)
    if kind == "sym":
        Y0 = P.sym_raw(Uraw, lam, X, compute=dt)
        Y, rec = P.sym_raw(Uraw, lam, X, compute=dt, save=True)
        dX, dU, dlam = P.sym_bwd_raw(Uraw, lam, X, G, compute=dt, saved=rec)
        dX0, dU0, dlam0 = P.sym_bwd_raw(Uraw, lam, X, G, compute=dt)
        rdX, rdU, rdlam = oracle.sym_bwd(host(Uraw), host(lam), host(X), host(G))
        m = 2 * (64 if h <= 64 else 128)
    else:
        tr = kind == "apply_T"
        Y0 = P.apply_raw(Uraw, X, trans=tr, compute=dt)
        Y, rec = P.apply_raw(Uraw, X, trans=tr, compute=dt, save=True)
        dX, dU = P.apply_bwd_raw(Uraw, X, G, trans=tr, compute=dt, saved=rec)
        dX0, dU0 = P.apply_bwd_raw(Uraw, X, G, trans=tr, compute=dt)
        rdX, rdU = oracle.apply_bwd(host(Uraw), host(X), host(G), trans=tr)
        m = 64 if h <= 64 else 128
    torch.cuda.synchronize()
    # writing the record leaves the forward's output unchanged, bit for bit
    assert torch.equal(Y, Y0)
    ldc = max(32, (N + 31) // 32 * 32)
    assert rec.numel() > m * ldc * 2
    cols = rec[:m * ldc * 2].view(torch.int16).view(m, ldc)
    assert torch.count_nonzero(cols[:, N:]) == 0
    # dX comes from the pass over dY alone
    assert torch.equal(dX, dX0)
    assert rel_rows(host(dX), rdX) < TOL16
    assert rel_fro(host(dU), rdU) < TOL16, rel_fro(host(dU), rdU)
    assert rel_refl(host(dU), rdU) < TOL16, rel_refl(host(dU), rdU)
    assert rel_fro(host(dU), host(dU0)) < 1e-2
    if kind == "sym":
        assert rel_fro(host(dlam), rdlam) < TOL16
        assert rel_fro(host(dlam), host(dlam0)) < 1e-2


def test_wy_saved_record_empty_batch():
    dt = torch.bfloat16
    n = 256
    U, _ = make(n, 6, 1, dt)
    E = torch.empty((0, n), dtype=dt, device=dev())
    # a freed, non-zero block that the record is likely to reuse
    rec0 = torch.full((1 << 16,), 7, dtype=torch.uint8, device=dev())
    del rec0
    Y, rec = P.apply_raw(U, E, compute=dt, save=True)
    torch.cuda.synchronize()
    assert Y.shape == (0, n) and rec.numel() > 64 * 32 * 2
    assert torch.count_nonzero(rec[:64 * 32 * 2]) == 0
    dX, dU = P.apply_bwd_raw(U, E, E, compute=dt, saved=rec)
    torch.cuda.synchronize()
    assert torch.count_nonzero(dU) == 0


def test_wy_autograd_uses_record():
    """apply/sym_apply keep the record when the reflectors need a gradient;
    the gradients still match the oracle."""
    dt = torch.float16
    n, h, N = 1024, 40, 96
    U, X = make(n, h, N, dt, seed=21)
    U.requires_grad_(True)
    G = torch.randn((N, n), device=dev()).to(dt)
    Y = P.apply(U, X, compute=dt)
    assert Y.grad_fn is not None
    (Y.float() * G.float()).sum().backward()
    _, rdU = oracle.apply_bwd(host(U), host(X), host(G))
    assert rel_fro(host(U.grad), rdU) < TOL16
    assert rel_refl(host(U.grad), rdU) < TOL16, rel_refl(host(U.grad), rdU)


@pytest.mark.parametrize("n,h,N", [(256, 12, 40), (8192, 64, 37)])  # resident / streaming kernel
def test_wy_saved_record_in_place(n, h, N):
    """A forward that keeps its record may overwrite its input (Y = X); the
    backward, given the original X, matches the plain backward."""
    dt = torch.bfloat16
    U, X = make(n, h, N, dt, seed=31)
    G = torch.randn((N, n), device=dev()).to(dt)
    Xi = X.clone()
    _, rec = P.apply_raw(U, Xi, compute=dt, out=Xi, save=True)
    ref = oracle.apply(host(U), host(X))
    assert rel_rows(host(Xi), ref) < TOL16
    dX, dU = P.apply_bwd_raw(U, X, G, compute=dt, saved=rec)
    rdX, rdU = oracle.apply_bwd(host(U), host(X), host(G))
    assert rel_rows(host(dX), rdX) < TOL16
    assert rel_fro(host(dU), rdU) < TOL16
    assert rel_refl(host(dU), rdU) < TOL16, rel_refl(host(dU), rdU)


# ----------------------------------------------------------------------------
# FP32 data on the WY path: rounded to the compute type, widened back
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("dname", ["bf16", "f16"])
@pytest.mark.parametrize("n,h,N", [(512, 9, 100), (8192, 64, 37)])  # resident / streaming kernel
def test_wy_fp32_data_equals_16bit_path(dname, n, h, N):
    """FP32 data gives exactly the 16-bit path's results on the rounded data,
    widened to FP32, forward and backward (with and without the saved record)."""
    dt = DT[dname]
    U, _ = make(n, h, N, dt, seed=41)
    Xf = torch.tensor(synth.gaussian((N, n), seed=42), dtype=torch.float32, device=dev())
    Gf = torch.tensor(synth.gaussian((N, n), seed=43, stream=synth.STREAM_G), dtype=torch.float32,
                      device=dev())
    lam = torch.tensor(synth.eig_loguniform(n, seed=5), dtype=torch.float32, device=dev())
    X16, G16 = Xf.to(dt), Gf.to(dt)
    for trans in (False, True):
        Y = P.apply_raw(U, Xf, trans=trans, compute=dt)
        assert Y.dtype == torch.float32
        assert torch.equal(Y, P.apply_raw(U, X16, trans=trans, compute=dt).float())
        dX, dU = P.apply_bwd_raw(U, Xf, Gf, trans=trans, compute=dt)
        dX16, dU16 = P.apply_bwd_raw(U, X16, G16, trans=trans, compute=dt)
        assert torch.equal(dX, dX16.float()) and torch.equal(dU, dU16)
    Y, rec = P.sym_raw(U, lam, Xf, compute=dt, save=True)
    Y16, rec16 = P.sym_raw(U, lam, X16, compute=dt, save=True)
    m = 2 * (64 if h <= 64 else 128)
    nb = m * max(32, (N + 31) // 32 * 32) * 2  # the coefficient rows of the record
    assert torch.equal(Y, Y16.float()) and torch.equal(rec[:nb], rec16[:nb])
    dX, dU, dl = P.sym_bwd_raw(U, lam, Xf, Gf, compute=dt, saved=rec)
    dX16, dU16, dl16 = P.sym_bwd_raw(U, lam, X16, G16, compute=dt, saved=rec16)
    assert torch.equal(dX, dX16.float()) and torch.equal(dU, dU16) and torch.equal(dl, dl16)
    # and against the oracle on the FP32 data (rounding of X is path error here)
    ref = oracle.sym(host(U), host(lam), host(Xf))
    assert rel_rows(host(Y), ref) < TOL16
