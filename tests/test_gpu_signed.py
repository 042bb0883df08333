"""Diagonals on either side of the fused forward ops (eq. 1: D times the
reflector product; Result 3: the product times D; eq. thesbar: D on both sides
of the symmetric form) through hh_forward_signed, against the FP64 oracle.

Shapes cover each lane layout of the fused kernel (16-lane rows, two vectors
per row, 64-lane vectors with 8-wave blocks, and the largest n, where the
diagonals push the block to the wide on-chip budget), ragged batches, and d in
{+1, -1}^n as the paper has it plus a general positive diagonal.  Tolerances as
the other fused parity tests: FP64 1e-12, FP32 1e-5 relative.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import rel_elem, rel_fro, rel_rows, rel_refl

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1811_07624_amd")
from paper_1811_07624_amd import _lib as L  # noqa: E402

DT = {"f64": torch.float64, "f32": torch.float32}
TOL = {"f64": 1e-12, "f32": 1e-5}
SHAPES = {"f64": [(100, 5, 333), (1000, 10, 257), (2048, 9, 130), (4096, 3, 70)],
          "f32": [(100, 5, 333), (1000, 10, 257), (2048, 9, 130), (8192, 3, 70)]}
MODES = ["in", "out", "both"]


def _dev():
    return torch.device("cuda:0")


def _host(t):
    return t.detach().to("cpu", torch.float64).numpy()


def _signs(n, seed):
    return np.where(synth.host_rng(seed, 11).random(n) < 0.5, -1.0, 1.0)


def _cases():
    out = []
    for t, shapes in SHAPES.items():
        for (n, h, N) in shapes:
            for op in ("apply", "apply_T", "sym"):
                for m in MODES:
                    out.append((t, op, m, n, h, N))
            out.append((t, "mahal", "in", n, h, N))
    return out


def _inputs(t, n, h, N, seed):
    dt = DT[t]
    U = torch.tensor(synth.reflectors(n, h, seed=seed), dtype=dt, device=_dev())
    lam = torch.tensor(synth.eig_uniform(n, seed=seed), dtype=dt, device=_dev())
    X = torch.tensor(synth.gaussian((N, n), seed=seed), dtype=dt, device=_dev())
    Xb = torch.tensor(synth.gaussian((N, n), seed=seed, stream=synth.STREAM_XB), dtype=dt, device=_dev())
    return U, lam, X, Xb


@pytest.mark.parametrize("t,op,mode,n,h,N", _cases(), ids=lambda v: str(v))
def test_signed_matches_oracle(t, op, mode, n, h, N):
    dt = DT[t]
    seed = n + h + N
    U, lam, X, Xb = _inputs(t, n, h, N, seed)
    d = _signs(n, seed)
    dd = torch.tensor(d, dtype=dt, device=_dev())
    din = dd if mode in ("in", "both") else None
    dout = dd if mode in ("out", "both") else None
    Y = P.signed_raw(op, U, X, d_in=din, d_out=dout, lam=lam if op in ("sym", "mahal") else None,
                     Xb=Xb if op == "mahal" else None)
    torch.cuda.synchronize()
    ref = oracle.signed(op, _host(U), _host(X), d_in=None if din is None else d,
                        d_out=None if dout is None else d, lam=_host(lam), Xb=_host(Xb))
    if op == "mahal":
        assert rel_elem(_host(Y), ref) < TOL[t]
    else:
        assert rel_rows(_host(Y), ref) < TOL[t]


@pytest.mark.parametrize("t", ["f64", "f32"])
def test_signed_general_diagonal(t):
    """Entries other than +-1 are applied as given (diag(d_out) Q diag(lam) Q^T diag(d_in))."""
    dt = DT[t]
    n, h, N = 520, 7, 100
    U, lam, X, _ = _inputs(t, n, h, N, 9)
    rng = synth.host_rng(9, 12)
    a, b = rng.uniform(0.5, 2.0, n), rng.uniform(0.5, 2.0, n)
    Y = P.signed_raw("sym", U, X, d_in=torch.tensor(a, dtype=dt, device=_dev()),
                     d_out=torch.tensor(b, dtype=dt, device=_dev()), lam=lam)
    ref = oracle.signed("sym", _host(U), _host(X), d_in=a, d_out=b, lam=_host(lam))
    assert rel_rows(_host(Y), ref) < TOL[t]


@pytest.mark.parametrize("t,n", [("f64", 64), ("f32", 1000), ("f32", 8192)])
def test_signed_unit_diagonal_is_plain_op_bitwise(t, n):
    """d = 1: the plain ops, bit for bit (multiplying by 1 is exact and the
    reflections run in the same order)."""
    dt = DT[t]
    h, N = 6, 77
    U, lam, X, Xb = _inputs(t, n, h, N, 3)
    one = torch.ones(n, dtype=dt, device=_dev())
    assert torch.equal(P.signed_raw("apply", U, X, d_in=one, d_out=one), P.apply_raw(U, X))
    assert torch.equal(P.signed_raw("apply_T", U, X, d_in=one, d_out=one), P.apply_raw(U, X, trans=True))
    assert torch.equal(P.signed_raw("sym", U, X, d_in=one, d_out=one, lam=lam), P.sym_raw(U, lam, X))
    assert torch.equal(P.signed_raw("mahal", U, X, d_in=one, lam=lam, Xb=Xb), P.mahal_raw(U, lam, X, Xb))


@pytest.mark.parametrize("t,n,h,tol", [("f64", 40, 17, 1e-12), ("f32", 256, 100, 1e-5)])
def test_signed_result3_identity_block(t, n, h, tol):
    """Eq. ReflectorStructure: with D = diag(sign of the top block, sign(diag U~)),
    D J_h ... J_1 U = [I_h 0; 0 D_1 U~] and D_1 U~ has a positive diagonal."""
    dt = DT[t]
    U0, _ = np.linalg.qr(np.random.default_rng(n + h).standard_normal((n, n)))
    V, _ = oracle.householder_qr(U0)
    Vh = V[:h]
    plain = oracle.apply(Vh, U0.T, trans=True).T
    d = np.concatenate([np.sign(np.diag(plain)[:h]), np.sign(np.diag(plain[h:, h:]))])
    X = torch.tensor(np.ascontiguousarray(U0.T), dtype=dt, device=_dev())
    B = _host(P.signed_raw("apply_T", torch.tensor(Vh, dtype=dt, device=_dev()), X,
                           d_out=torch.tensor(d, dtype=dt, device=_dev()))).T
    assert np.abs(B[:h, :h] - np.eye(h)).max() < tol
    assert np.abs(B[:h, h:]).max() < tol and np.abs(B[h:, :h]).max() < tol
    assert np.all(np.diag(B[h:, h:]) > 0)


def test_signed_in_place_and_empty():
    n, h, N = 300, 4, 50
    U, lam, X, _ = _inputs("f32", n, h, N, 4)
    d = torch.tensor(_signs(n, 4), dtype=torch.float32, device=_dev())
    ref = P.signed_raw("sym", U, X, d_in=d, d_out=d, lam=lam)
    Xc = X.clone()
    P.signed_raw("sym", U, Xc, d_in=d, d_out=d, lam=lam, out=Xc)
    assert torch.equal(Xc, ref)
    E = torch.empty((0, n), dtype=torch.float32, device=_dev())
    assert P.signed_raw("apply", U, E, d_out=d).shape == (0, n)


def test_signed_rejected_on_wy_and_for_distance_output():
    n, h, N = 256, 8, 32
    U = torch.tensor(synth.reflectors(n, h, seed=1), dtype=torch.float32, device=_dev())
    X = torch.zeros((N, n), dtype=torch.bfloat16, device=_dev())
    d = torch.ones(n, dtype=torch.float32, device=_dev())
    with pytest.raises(L.HHError) as e:
        P.signed_raw("apply", U, X, d_in=d)
    assert e.value.status == L.HH_ERR_UNSUPPORTED
    Xf = torch.zeros((N, n), dtype=torch.float32, device=_dev())
    with pytest.raises(L.HHError) as e:
        P.signed_raw("mahal", U, Xf, d_out=d, lam=d, Xb=Xf)
    assert e.value.status == L.HH_ERR_INVALID_ARG


# ---------------------------------------------------------------------------
# gradients (hh_backward_signed)

GTOL = {"f64": 1e-10, "f32": 1e-5}
BSHAPES = {"f64": [(100, 5, 333), (1000, 6, 257)],
           "f32": [(100, 5, 333), (1000, 10, 257), (2048, 4, 130)]}


def _bcases():
    out = []
    for t, shapes in BSHAPES.items():
        for (n, h, N) in shapes:
            for op in ("apply", "apply_T", "sym"):
                for m in MODES:
                    out.append((t, op, m, n, h, N))
            out.append((t, "mahal", "in", n, h, N))
    return out


@pytest.mark.parametrize("t,op,mode,n,h,N", _bcases(), ids=lambda v: str(v))
def test_signed_bwd_matches_oracle(t, op, mode, n, h, N):
    dt = DT[t]
    seed = 7 * n + h + N
    U, lam, X, Xb = _inputs(t, n, h, N, seed)
    d = _signs(n, seed)
    dd = torch.tensor(d, dtype=dt, device=_dev())
    din = dd if mode in ("in", "both") else None
    dout = dd if mode in ("out", "both") else None
    Uh, lh, Xh, Xbh = _host(U), _host(lam), _host(X), _host(Xb)
    if op == "mahal":
        w = torch.tensor(synth.gaussian(N, seed=seed, stream=synth.STREAM_W), dtype=dt, device=_dev())
        dXa, dXb, dU, dl = P.signed_bwd_raw(op, U, X, w, d_in=din, lam=lam, Xb=Xb)
        torch.cuda.synchronize()
        r = oracle.signed_bwd(op, Uh, Xh, _host(w), d_in=d, lam=lh, Xb=Xbh)
        assert rel_rows(_host(dXa), r[0]) < GTOL[t]
        assert rel_rows(_host(dXb), r[1]) < GTOL[t]
        assert rel_fro(_host(dU), r[2]) < GTOL[t]
        assert rel_refl(_host(dU), r[2]) < GTOL[t], rel_refl(_host(dU), r[2])
        assert rel_fro(_host(dl), r[3]) < GTOL[t]
        return
    G = torch.tensor(synth.gaussian((N, n), seed=seed, stream=synth.STREAM_G), dtype=dt, device=_dev())
    dX, dU, dl = P.signed_bwd_raw(op, U, X, G, d_in=din, d_out=dout, lam=lam if op == "sym" else None)
    torch.cuda.synchronize()
    r = oracle.signed_bwd(op, Uh, Xh, _host(G), d_in=None if din is None else d,
                          d_out=None if dout is None else d, lam=lh)
    assert rel_rows(_host(dX), r[0]) < GTOL[t]
    assert rel_fro(_host(dU), r[1]) < GTOL[t]
    assert rel_refl(_host(dU), r[1]) < GTOL[t], rel_refl(_host(dU), r[1])
    if op == "sym":
        assert rel_fro(_host(dl), r[2]) < GTOL[t]


@pytest.mark.parametrize("t", ["f64", "f32"])
def test_signed_bwd_unit_diagonal_is_plain_bwd_bitwise(t):
    dt = DT[t]
    n, h, N = 1000, 6, 200
    U, lam, X, Xb = _inputs(t, n, h, N, 8)
    G = torch.tensor(synth.gaussian((N, n), seed=8, stream=synth.STREAM_G), dtype=dt, device=_dev())
    one = torch.ones(n, dtype=dt, device=_dev())
    a = P.signed_bwd_raw("sym", U, X, G, d_in=one, d_out=one, lam=lam)
    b = P.sym_bwd_raw(U, lam, X, G)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    a = P.signed_bwd_raw("apply_T", U, X, G, d_in=one, d_out=one)
    b = P.apply_bwd_raw(U, X, G, trans=True)
    for x, y in zip(a[:2], b):
        assert torch.equal(x, y)


def test_signed_bwd_rejected_on_wy():
    n, h, N = 256, 8, 32
    U = torch.tensor(synth.reflectors(n, h, seed=1), dtype=torch.float32, device=_dev())
    X = torch.zeros((N, n), dtype=torch.bfloat16, device=_dev())
    d = torch.ones(n, dtype=torch.float32, device=_dev())
    with pytest.raises(L.HHError) as e:
        P.signed_bwd_raw("apply", U, X, X, d_out=d)
    assert e.value.status == L.HH_ERR_UNSUPPORTED


@pytest.mark.parametrize("op", ["apply", "apply_T", "sym", "mahal"])
def test_signed_autograd(op):
    """torch autograd through the signed forward gives the oracle's gradients."""
    t, n, h, N = "f64", 200, 5, 60
    dt = DT[t]
    U, lam, X, Xb = _inputs(t, n, h, N, 21)
    d = _signs(n, 21)
    dd = torch.tensor(d, dtype=dt, device=_dev())
    U.requires_grad_(True)
    X.requires_grad_(True)
    lam.requires_grad_(op in ("sym", "mahal"))
    Xb.requires_grad_(op == "mahal")
    dout = None if op == "mahal" else dd
    Y = P.signed(op, U, X, d_in=dd, d_out=dout, lam=lam if op in ("sym", "mahal") else None,
                 Xb=Xb if op == "mahal" else None)
    if op == "mahal":
        w = torch.tensor(synth.gaussian(N, seed=21, stream=synth.STREAM_W), dtype=dt, device=_dev())
    else:
        w = torch.tensor(synth.gaussian((N, n), seed=21, stream=synth.STREAM_G), dtype=dt, device=_dev())
    (Y * w).sum().backward()
    r = oracle.signed_bwd(op, _host(U), _host(X), _host(w), d_in=d, d_out=None if dout is None else d,
                          lam=_host(lam), Xb=_host(Xb))
    if op == "mahal":
        assert rel_rows(_host(X.grad), r[0]) < GTOL[t]
        assert rel_rows(_host(Xb.grad), r[1]) < GTOL[t]
        assert rel_fro(_host(U.grad), r[2]) < GTOL[t]
        assert rel_refl(_host(U.grad), r[2]) < GTOL[t], rel_refl(_host(U.grad), r[2])
        assert rel_fro(_host(lam.grad), r[3]) < GTOL[t]
    else:
        assert rel_rows(_host(X.grad), r[0]) < GTOL[t]
        assert rel_fro(_host(U.grad), r[1]) < GTOL[t]
        assert rel_refl(_host(U.grad), r[1]) < GTOL[t], rel_refl(_host(U.grad), r[1])
        if op == "sym":
            assert rel_fro(_host(lam.grad), r[2]) < GTOL[t]


@pytest.mark.parametrize("t", ["f64", "f32"])
def test_signed_edge_cases(t):
    """h = 0 leaves only the diagonals (exact products); an empty batch gives
    zero dU and dlam."""
    dt = DT[t]
    n, N = 129, 37
    rng = synth.host_rng(31, 13)
    a = torch.tensor(rng.uniform(0.5, 2.0, n), dtype=dt, device=_dev())
    b = torch.tensor(rng.uniform(0.5, 2.0, n), dtype=dt, device=_dev())
    X = torch.tensor(synth.gaussian((N, n), seed=31), dtype=dt, device=_dev())
    U0 = torch.empty((0, n), dtype=dt, device=_dev())
    lam = torch.tensor(synth.eig_uniform(n, seed=31), dtype=dt, device=_dev())
    assert torch.equal(P.signed_raw("apply", U0, X, d_in=a, d_out=b), X * a * b)
    assert torch.equal(P.signed_raw("sym", U0, X, d_in=a, d_out=b, lam=lam), X * a * lam * b)
    U = torch.tensor(synth.reflectors(n, 4, seed=31), dtype=dt, device=_dev())
    E = torch.empty((0, n), dtype=dt, device=_dev())
    dX, dU, dl = P.signed_bwd_raw("sym", U, E, E, d_in=a, d_out=b, lam=lam)
    torch.cuda.synchronize()
    assert dX.shape == (0, n) and torch.count_nonzero(dU) == 0 and torch.count_nonzero(dl) == 0


@pytest.mark.parametrize("op", ["apply", "sym", "mahal"])
def test_signed_autograd_only_needed_grads(op):
    """Only the gradients autograd asks for are computed: with just U
    requiring a gradient, dU matches the full backward's and X gets none."""
    t = "f32"
    dt = DT[t]
    n, h, N = 300, 5, 64
    U, lam, X, Xb = _inputs(t, n, h, N, 21)
    d = torch.tensor(_signs(n, 21), dtype=dt, device=_dev())
    Ug = U.clone().requires_grad_(True)
    kw = dict(d_in=d, lam=lam if op in ("sym", "mahal") else None, Xb=Xb if op == "mahal" else None)
    if op != "mahal":
        kw["d_out"] = d
    Y = P.signed(op, Ug, X, **kw)
    G = torch.tensor(synth.gaussian(tuple(Y.shape), seed=21, stream=synth.STREAM_G), dtype=dt,
                     device=_dev())
    (Y * G).sum().backward()
    full = P.signed_bwd_raw(op, U, X, G, **kw)
    dU_full = full[2] if op == "mahal" else full[1]
    torch.cuda.synchronize()
    assert X.grad is None
    assert rel_fro(_host(Ug.grad), _host(dU_full)) < 1e-6
