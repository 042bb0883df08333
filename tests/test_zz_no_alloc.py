"""hh_forward_noalloc: the forward ops with the library's static device scratch
in place of a workspace argument, for callers that cannot allocate.

Each case calls the entry point through the C ABI twice in a row, the second
time on a smaller batch (the scratch keeps the first call's contents), and
compares both outputs with the entry point that takes a workspace (same
kernels on the same inputs: bit for bit) and with the FP64 oracle at the
stated tolerances.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import rel_elem, rel_rows

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1811_07624_amd")
from paper_1811_07624_amd import _lib as L  # noqa: E402

TOL = {torch.float64: 1e-12, torch.float32: 1e-5, torch.bfloat16: 2e-2, torch.float16: 2e-2}


def dev():
    return torch.device("cuda:0")


def host(t):
    return t.detach().to("cpu", torch.float64).numpy()


def _data(n, h, N, dt, pdt, seed):
    U = torch.tensor(synth.reflectors(n, h, seed=seed), dtype=pdt, device=dev())
    lam = torch.tensor(synth.eig_uniform(n, seed=seed), dtype=pdt, device=dev())
    X = torch.tensor(synth.gaussian((N, n), seed=seed), dtype=torch.float32, device=dev()).to(dt)
    Xb = torch.tensor(synth.gaussian((N, n), seed=seed, stream=synth.STREAM_XB),
                      dtype=torch.float32, device=dev()).to(dt)
    return U, lam, X, Xb


CASES = [
    # (op, n, h, (N1, N2), data dtype, compute dtype)
    ("apply", 4096, 64, (3000, 700), torch.bfloat16, torch.bfloat16),     # resident WY kernel
    ("apply_T", 8192, 128, (600, 130), torch.float16, torch.float16),     # streaming WY kernel
    ("sym", 8192, 128, (520, 33), torch.float16, torch.float16),
    ("sym", 1024, 10, (5000, 1000), torch.float32, torch.float32),        # fused FP32
    ("mahal", 512, 9, (4000, 257), torch.float32, torch.float32),
    ("apply", 64, 4, (1024, 100), torch.float64, torch.float64),          # fused FP64
    ("apply", 1024, 64, (300, 45), torch.float32, torch.bfloat16),        # WY with FP32 data
]


def _reference(op, U, lam, X, Xb, comp):
    if op == "apply":
        return P.apply_raw(U, X, compute=comp)
    if op == "apply_T":
        return P.apply_raw(U, X, trans=True, compute=comp)
    if op == "sym":
        return P.sym_raw(U, lam, X, compute=comp)
    return P.mahal_raw(U, lam, X, Xb, compute=comp)


def _oracle(op, U, lam, X, Xb):
    if op in ("apply", "apply_T"):
        return oracle.apply(host(U), host(X), trans=op == "apply_T")
    if op == "sym":
        return oracle.sym(host(U), host(lam), host(X))
    return oracle.mahal(host(U), host(lam), host(X), host(Xb))


@pytest.mark.parametrize("op,n,h,Ns,dt,comp", CASES)
def test_noalloc_matches_workspace_entry_point(op, n, h, Ns, dt, comp):
    pdt = comp if comp in (torch.float64, torch.float32) else torch.float32
    U, lam, X, Xb = _data(n, h, Ns[0], dt, pdt, seed=n + h)
    for N in Ns:  # two calls in a row, the second on a smaller batch
        Xs, Xbs = X[:N], Xb[:N]
        print(f"noalloc {op} n={n} h={h} N={N} {dt} -> {comp}", flush=True)
        Y = P.forward_noalloc_raw(op, U, Xs, lam=lam if op in ("sym", "mahal") else None,
                                  Xb=Xbs if op == "mahal" else None, compute=comp)
        R = _reference(op, U, lam, Xs, Xbs, comp)
        torch.cuda.synchronize()
        assert torch.equal(Y, R), (op, N)
        ref = _oracle(op, U, lam, Xs, Xbs)
        err = rel_elem(host(Y), ref) if op == "mahal" else rel_rows(host(Y), ref)
        assert err < TOL[comp], (op, N, err)


def test_noalloc_in_place_and_empty():
    n, h = 2048, 32
    U, lam, X, _ = _data(n, h, 400, torch.bfloat16, torch.float32, seed=5)
    R = P.apply_raw(U, X, compute=torch.bfloat16)
    Xi = X.clone()
    P.forward_noalloc_raw("apply", U, Xi, compute=torch.bfloat16, out=Xi)
    E = X[:0]
    assert P.forward_noalloc_raw("apply", U, E, compute=torch.bfloat16).shape == (0, n)
    torch.cuda.synchronize()
    assert torch.equal(Xi, R)


def test_noalloc_rejects_oversized_scratch():
    """A call whose workspace exceeds the static scratch is refused before
    anything is enqueued, and the output is left untouched."""
    n, h, N = 4096, 64, 4096  # FP32 data on the WY path: 16-bit copies of X and Y, 64 MiB
    U = torch.tensor(synth.reflectors(n, h, seed=1), dtype=torch.float32, device=dev())
    X = torch.zeros((N, n), dtype=torch.float32, device=dev())
    Y = torch.full((N, n), 7.0, dtype=torch.float32, device=dev())
    with pytest.raises(L.HHError) as ei:
        P.forward_noalloc_raw("apply", U, X, compute=torch.bfloat16, out=Y)
    assert ei.value.status == L.HH_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert bool((Y == 7.0).all())
    desc = L.make_desc(n, h, N, torch.float32, torch.float32, torch.bfloat16)
    need = ctypes.c_size_t(0)
    assert L.lib().hh_workspace_size(L.HH_OP_APPLY, ctypes.byref(desc), ctypes.byref(need)) == 0
    assert need.value > L.NOALLOC_SCRATCH_BYTES
