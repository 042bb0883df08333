"""Seeded random shapes through both kernel families against the FP64 oracle.

Each case draws (n, h, N), an operation and a number type from a fixed seed, so
the set of cases is the same on every run; shapes the library rejects as
unsupported (e.g. a fused backward whose reflectors do not fit on chip) are
skipped, never silently handled on the host.  Tolerances as in the other
parity tests: FP64 1e-12 (outputs) / 1e-10 (gradients), FP32 1e-5, 16-bit 2e-2,
the last scaled by max(1, sqrt(h / n)): with more reflectors than dimensions
every direction is reflected about h / n times by 16-bit reflector vectors,
whose rounding errors add up like a random walk (BF16 at n = 8, h = 83 gives
2.2e-2).
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

DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}
TOL = {"f64": (1e-12, 1e-10), "f32": (1e-5, 1e-5), "bf16": (2e-2, 2e-2), "f16": (2e-2, 2e-2)}
OPS = ["apply", "apply_T", "sym", "mahal"]


def _cases():
    rng = np.random.default_rng(20261202)
    out = []
    for i in range(24):  # fused kernels
        t = "f64" if i % 2 == 0 else "f32"
        n = int(np.exp(rng.uniform(0, np.log(4096))))
        h = int(rng.integers(0, 41))
        N = int(rng.integers(0, 301))
        out.append(("fused", t, OPS[i % 4], n, h, N, i))
    for i in range(16):  # compact-WY kernels
        t = "bf16" if i % 2 == 0 else "f16"
        n = 8 * int(np.exp(rng.uniform(0, np.log(1024))))
        h = int(rng.integers(0, 129))
        N = int(rng.integers(0, 201))
        out.append(("wy", t, OPS[i % 3], n, h, N, 100 + i))
    return out


def _dev():
    return torch.device("cuda:0")


def _host(t):
    return t.detach().to("cpu", torch.float64).numpy()


def _unsupported(e):
    return isinstance(e, L.HHError) and e.status == L.HH_ERR_UNSUPPORTED


@pytest.mark.parametrize("algo,tname,op,n,h,N,seed", _cases(),
                         ids=lambda v: str(v))
def test_random_shape(algo, tname, op, n, h, N, seed):
    dt = DT[tname]
    ytol, gtol = TOL[tname]
    if algo == "wy":
        scale = max(1.0, float(np.sqrt(h / n)))
        ytol, gtol = ytol * scale, gtol * scale
    pdt = torch.float64 if dt == torch.float64 else torch.float32
    U = torch.tensor(synth.reflectors(n, h, seed=seed), dtype=pdt, device=_dev())
    U = U * torch.tensor(synth.host_rng(seed, 7).uniform(0.5, 2.0, (h, 1)), dtype=pdt, device=_dev())
    lam = torch.tensor(synth.eig_uniform(n, seed=seed), dtype=pdt, device=_dev())
    X = torch.tensor(synth.gaussian((N, n), seed=seed), dtype=torch.float32 if dt != torch.float64 else dt,
                     device=_dev()).to(dt)
    G = torch.tensor(synth.gaussian((N, n), seed=seed, stream=synth.STREAM_G),
                     dtype=torch.float32 if dt != torch.float64 else dt, device=_dev()).to(dt)
    Uh, lh, Xh, Gh = _host(U), _host(lam), _host(X), _host(G)
    try:
        if op in ("apply", "apply_T"):
            tr = op == "apply_T"
            Y = P.apply_raw(U, X, trans=tr, compute=dt)
            dX, dU = P.apply_bwd_raw(U, X, G, trans=tr, compute=dt)
            torch.cuda.synchronize()
            rdX, rdU = oracle.apply_bwd(Uh, Xh, Gh, trans=tr)
            assert rel_rows(_host(Y), oracle.apply(Uh, Xh, trans=tr)) < ytol
            assert rel_rows(_host(dX), rdX) < gtol
            if N > 0 and h > 0:
                assert rel_fro(_host(dU), rdU) < gtol
                assert rel_refl(_host(dU), rdU) < gtol, rel_refl(_host(dU), rdU)
        elif op == "sym":
            Y = P.sym_raw(U, lam, X, compute=dt)
            dX, dU, dl = P.sym_bwd_raw(U, lam, X, G, compute=dt)
            torch.cuda.synchronize()
            rdX, rdU, rdl = oracle.sym_bwd(Uh, lh, Xh, Gh)
            assert rel_rows(_host(Y), oracle.sym(Uh, lh, Xh)) < ytol
            assert rel_rows(_host(dX), rdX) < gtol
            if N > 0:
                assert rel_fro(_host(dl), rdl) < gtol
                if h > 0:
                    assert rel_fro(_host(dU), rdU) < gtol
                    assert rel_refl(_host(dU), rdU) < gtol, rel_refl(_host(dU), rdU)
        else:
            Xb = torch.tensor(synth.gaussian((N, n), seed=seed, stream=synth.STREAM_XB), dtype=dt,
                              device=_dev())
            w = torch.tensor(synth.gaussian(N, seed=seed, stream=synth.STREAM_W), dtype=pdt, device=_dev())
            d = P.mahal_raw(U, lam, X, Xb)
            dXa, dXb, dU, dl = P.mahal_bwd_raw(U, lam, X, Xb, w)
            torch.cuda.synchronize()
            Xbh = _host(Xb)
            assert rel_elem(_host(d), oracle.mahal(Uh, lh, Xh, Xbh)) < ytol
            rdXa, rdXb, rdU, rdl = oracle.mahal_bwd(Uh, lh, Xh, Xbh, _host(w))
            assert rel_rows(_host(dXa), rdXa) < gtol
            if N > 0:
                assert rel_fro(_host(dl), rdl) < gtol
                if h > 0:
                    assert rel_fro(_host(dU), rdU) < gtol
                    assert rel_refl(_host(dU), rdU) < gtol, rel_refl(_host(dU), rdU)
            if algo == "fused":  # the same through the record of dot products
                d2, rec = P.mahal_raw(U, lam, X, Xb, save=True)
                dXa2, _, dU2, dl2 = P.mahal_bwd_raw(U, lam, X, Xb, w, saved=rec)
                torch.cuda.synchronize()
                assert torch.equal(d2, d)
                assert rel_rows(_host(dXa2), rdXa) < gtol
                if N > 0:
                    assert rel_fro(_host(dl2), rdl) < gtol
                    if h > 0:
                        assert rel_fro(_host(dU2), rdU) < gtol
                        assert rel_refl(_host(dU2), rdU) < gtol, rel_refl(_host(dU2), rdU)
    except L.HHError as e:
        if _unsupported(e):
            pytest.skip(f"unsupported by the library: {e}")
        raise
