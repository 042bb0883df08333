"""Parity at the benchmark workloads' full sizes, in the launch configuration
the benchmark times, on sampled outputs the FP64 oracle computes one by one.

Inputs are drawn as the benchmark draws them (seeded reflectors and spectra on
the host, data by torch's generator on the device); the oracle gets the sampled
vectors' exact bits.  Gradients dU and dlam are sums over all N vectors, which
the oracle cannot redo at full size in seconds: the upstream gradient is set to
zero except on the sampled vectors.  The kernels still run the full batch (all
tiles, all reduction splits) and the sums then hold the sampled vectors' terms
only (every term of dU and dlam carries a factor of the upstream gradient), so
the oracle's gradient over the sampled vectors is the exact reference.
Tolerances: FP32 1e-5, BF16 and FP16 2e-2 relative.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import rel_elem, rel_fro, rel_rows, rel_refl

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1811_07624_amd")

TOL32, TOL16 = 1e-5, 2e-2


def dev():
    return torch.device("cuda:0")


def host(t):
    return t.detach().to("cpu", torch.float64).numpy()


def sample_idx(N, seed=0, k=32):
    """First and last 16 vectors and k seeded ones in between (sorted, unique)."""
    rng = np.random.default_rng(seed)
    idx = set(range(16)) | set(range(N - 16, N)) | set(rng.integers(0, N, k).tolist())
    return torch.tensor(sorted(idx), dtype=torch.long, device=dev())


def sparse_rows(N, n, idx, dtype, seed):
    """An (N, n) upstream gradient that is zero except on the rows idx."""
    G = torch.zeros((N, n), dtype=dtype, device=dev())
    vals = synth.gaussian((len(idx), n), seed=seed, stream=synth.STREAM_G)
    G[idx] = torch.tensor(vals, dtype=torch.float32, device=dev()).to(dtype)
    return G


def release():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_full_sym_fused_fp32():
    """Q diag(lam) Q^T X, n=1024, h=10, N=2^20, fused FP32."""
    n, h, N = 1024, 10, 1 << 20
    U = torch.tensor(synth.reflectors(n, h, seed=0), dtype=torch.float32, device=dev())
    lam = torch.tensor(synth.eig_uniform(n, seed=0), dtype=torch.float32, device=dev())
    X = synth.device_gaussian((N, n), seed=0, stream=synth.STREAM_X, device=dev())
    Y = P.sym_raw(U, lam, X)
    idx = sample_idx(N)
    ref = oracle.sym(host(U), host(lam), host(X[idx]))
    assert rel_rows(host(Y[idx]), ref) < TOL32
    # lam = c everywhere: S = c I, at full size
    Y = P.sym_raw(U, torch.full_like(lam, 3.0), X, out=Y)
    err = ((Y - 3.0 * X).norm(dim=1) / (3.0 * X).norm(dim=1)).max().item()
    assert err < TOL32
    del X, Y
    release()


def test_full_mahal_fused_fp32_fwd_bwd():
    """Distances and their gradients to U and lam, n=512, h=9, N=2^22 pairs, fused FP32."""
    n, h, N = 512, 9, 1 << 22
    U = torch.tensor(synth.reflectors(n, h, seed=0), dtype=torch.float32, device=dev())
    lam = torch.tensor(synth.eig_uniform(n, seed=0), dtype=torch.float32, device=dev())
    Xa = synth.device_gaussian((N, n), seed=0, stream=synth.STREAM_X, device=dev())
    Xb = synth.device_gaussian((N, n), seed=0, stream=synth.STREAM_XB, device=dev())
    d = P.mahal_raw(U, lam, Xa, Xb)
    idx = sample_idx(N, seed=1)
    Uh, lh, xa, xb = host(U), host(lam), host(Xa[idx]), host(Xb[idx])
    assert rel_elem(host(d[idx]), oracle.mahal(Uh, lh, xa, xb)) < TOL32
    w = torch.zeros(N, dtype=torch.float32, device=dev())
    w[idx] = torch.tensor(synth.gaussian(len(idx), seed=2, stream=synth.STREAM_W), dtype=torch.float32,
                          device=dev())
    _, _, dU, dlam = P.mahal_bwd_raw(U, lam, Xa, Xb, w, need_dX=False)
    _, _, rdU, rdlam = oracle.mahal_bwd(Uh, lh, xa, xb, host(w[idx]))
    assert rel_fro(host(dU), rdU) < TOL32
    assert rel_refl(host(dU), rdU) < TOL32, rel_refl(host(dU), rdU)
    assert rel_fro(host(dlam), rdlam) < TOL32
    del Xa, Xb
    release()


def test_full_qx_wy_bf16_fwd_bwd():
    """Q X, n=4096, h=64, N=2^18: compact-WY BF16 forward with its saved record
    and backward, and the fused FP32 forward on the same data."""
    n, h, N = 4096, 64, 1 << 18
    dt = torch.bfloat16
    U = torch.tensor(synth.reflectors(n, h, seed=0), dtype=torch.float32, device=dev())
    X = synth.device_gaussian((N, n), seed=0, stream=synth.STREAM_X, device=dev(), dtype=dt)
    Y, rec = P.apply_raw(U, X, compute=dt, save=True)
    idx = sample_idx(N, seed=3)
    Uh, xs = host(U), host(X[idx])
    ref = oracle.apply(Uh, xs)
    assert rel_rows(host(Y[idx]), ref) < TOL16
    del Y
    Xf = X.float()
    Yf = P.apply_raw(U, Xf)
    assert rel_rows(host(Yf[idx]), ref) < TOL32
    del Xf, Yf
    G = sparse_rows(N, n, idx, dt, seed=4)
    dX, dU = P.apply_bwd_raw(U, X, G, compute=dt, saved=rec)
    rdX, rdU = oracle.apply_bwd(Uh, xs, host(G[idx]))
    assert rel_rows(host(dX[idx]), rdX) < TOL16
    assert rel_fro(host(dU), rdU) < TOL16
    assert rel_refl(host(dU), rdU) < TOL16, rel_refl(host(dU), rdU)
    # dX = Q^T G: rows with G = 0 are exactly zero
    mask = torch.ones(N, dtype=torch.bool, device=dev())
    mask[idx] = False
    assert torch.count_nonzero(dX[mask]) == 0
    del X, G, dX, rec
    release()


def test_full_sym_wy_fp16_fwd_bwd():
    """Q diag(lam) Q^T X, n=8192, h=128, N=2^16, compact-WY FP16, forward with its
    saved record and backward to X, U and lam."""
    n, h, N = 8192, 128, 1 << 16
    dt = torch.float16
    U = torch.tensor(synth.reflectors(n, h, seed=0), dtype=torch.float32, device=dev())
    lam = torch.tensor(synth.eig_loguniform(n, seed=0), dtype=torch.float32, device=dev())
    X = synth.device_gaussian((N, n), seed=0, stream=synth.STREAM_X, device=dev(), dtype=dt)
    Y, rec = P.sym_raw(U, lam, X, compute=dt, save=True)
    idx = sample_idx(N, seed=5)
    Uh, lh, xs = host(U), host(lam), host(X[idx])
    assert rel_rows(host(Y[idx]), oracle.sym(Uh, lh, xs)) < TOL16
    del Y
    G = sparse_rows(N, n, idx, dt, seed=6)
    dX, dU, dlam = P.sym_bwd_raw(U, lam, X, G, compute=dt, saved=rec)
    rdX, rdU, rdlam = oracle.sym_bwd(Uh, lh, xs, host(G[idx]))
    assert rel_rows(host(dX[idx]), rdX) < TOL16
    assert rel_fro(host(dU), rdU) < TOL16
    assert rel_refl(host(dU), rdU) < TOL16, rel_refl(host(dU), rdU)
    assert rel_fro(host(dlam), rdlam) < TOL16
    del X, G, dX, rec
    release()


def _row_rel(A, B, chunk=1 << 15):
    """max over rows of ||a_j - b_j|| / ||b_j||, formed on the GPU in FP32
    chunk by chunk (a checker over every vector of a full batch)."""
    worst = 0.0
    for s in range(0, A.shape[0], chunk):
        a, b = A[s:s + chunk].float(), B[s:s + chunk].float()
        r = torch.linalg.vector_norm(a - b, dim=1) / torch.linalg.vector_norm(b, dim=1)
        worst = max(worst, float(r.max()))
    return worst


def _norm_dev(A, B, chunk=1 << 15):
    """max over rows of | ||a_j|| - ||b_j|| | / ||b_j|| (GPU, FP32)."""
    worst = 0.0
    for s in range(0, A.shape[0], chunk):
        na = torch.linalg.vector_norm(A[s:s + chunk].float(), dim=1)
        nb = torch.linalg.vector_norm(B[s:s + chunk].float(), dim=1)
        worst = max(worst, float(((na - nb).abs() / nb).max()))
    return worst


@pytest.mark.parametrize("n,h,N,dname", [(4096, 64, 1 << 18, "bf16"), (8192, 128, 1 << 16, "f16")])
def test_full_wy_every_vector(n, h, N, dname):
    """Invariants over every vector of the full batch (no oracle needed, so no
    tile escapes the check): Q preserves each vector's norm, within the
    output tolerance (| ||y|| - ||x|| | <= ||y^ - y||), and Q^T (Q x) = x
    within twice it (two applications)."""
    dt = {"bf16": torch.bfloat16, "f16": torch.float16}[dname]
    U = torch.tensor(synth.reflectors(n, h, seed=0), dtype=torch.float32, device=dev())
    X = synth.device_gaussian((N, n), seed=0, stream=synth.STREAM_X, device=dev(), dtype=dt)
    Y = P.apply_raw(U, X, compute=dt)
    assert _norm_dev(Y, X) < TOL16
    Z = P.apply_raw(U, Y, trans=True, compute=dt)
    assert _row_rel(Z, X) < 2 * TOL16
    del Y, Z
    # the symmetric form with lam = c everywhere is c X for every vector
    lam = torch.full((n,), 3.0, dtype=torch.float32, device=dev())
    S = P.sym_raw(U, lam, X, compute=dt)
    assert _row_rel(S, 3.0 * X.float()) < TOL16
    del X, S
    release()
