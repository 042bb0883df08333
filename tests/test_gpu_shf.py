"""GPU parity of SHF / SHF-SU (Algorithm 1, hh_shf) against the FP64 oracle
(oracle/shf.py), through the C ABI.

Both sides take the same decisions (the readings stated in the oracle: line
searches on the same grid with the same golden-section steps, the same
Kronecker sign rule and D rule, the same stopping tests), so the error after
the initialisation and after every sweep agrees up to rounding (relative
1e-6), and so do the sign diagonal and the approximation Sbar.  The
descent stops once a step gains less than 1e-12 of C; near a minimum C is
flat to second order, so the parameters themselves (spectrum, reflector
lines) are fixed only to about sqrt(1e-12) = 1e-6 of their scale by that
test, and rounding-level differences move them that much: they are
compared at 1e-5 of their scale.
Eigenvector signs differ between the two eigensolvers; the searches cover
both orientations, so the reflectors agree as lines (u u^T).  Sbar is then
applied to vectors by the transform kernels (the symmetric form with d on
both sides) and compared with the dense D U diag(sbar) U^T D.
"""
import numpy as np
import pytest
import torch

from oracle import shf as H
from tests._util import rel_rows

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1811_07624_amd")


def dev():
    return torch.device("cuda:0")


def rand_sym(n, seed):
    X = np.random.default_rng(seed).standard_normal((n, n))
    return (X + X.T) / 2


@pytest.mark.parametrize("n,h,K,su", [(16, 2, 6, False), (16, 2, 6, True), (33, 4, 6, True),
                                      (40, 3, 5, False), (64, 6, 4, True)])
def test_shf_matches_oracle(n, h, K, su):
    S = rand_sym(n, n + h)
    R, sb, d, err = P.shf(torch.tensor(S, device=dev()), h, K, spectrum_update=su)
    torch.cuda.synchronize()
    R, sb, d, err = (t.cpu().numpy() for t in (R, sb, d, err))
    Ur, sbr, dr, er = H.shf(S, h, K, spectrum_update=su)
    er = np.array(er)
    assert np.allclose(err[: len(er)], er, rtol=1e-6, atol=0)
    assert (err[len(er):] == err[len(er) - 1]).all()  # repeated once stopped
    assert (np.diff(err) <= 1e-9 * err[:-1]).all()  # monotone after the initialisation
    assert np.abs(sb - sbr).max() < 1e-5 * np.abs(sbr).max()
    assert (d == dr).all()
    for k in range(h):
        assert np.abs(np.outer(R[k], R[k]) - np.outer(Ur[k], Ur[k])).max() < 1e-5
    Sb = H.approx(sb, d, R)
    assert np.linalg.norm(Sb - H.approx(sbr, dr, Ur)) < 1e-6 * np.linalg.norm(S)
    assert abs(np.linalg.norm(S - Sb) ** 2 - err[-1]) < 1e-9 * err[-1]
    # Sbar through the transform kernels
    X = np.random.default_rng(7).standard_normal((50, n))
    t = lambda a: torch.tensor(a, device=dev())
    Y = P.signed_raw("sym", t(R), t(X), d_in=t(d), d_out=t(d), lam=t(sb)).cpu().numpy()
    assert rel_rows(Y, X @ Sb) < 1e-12


def test_shf_one_reflector_exact():
    n = 24
    rng = np.random.default_rng(1)
    u = rng.standard_normal(n)
    u /= np.linalg.norm(u)
    s = rng.standard_normal(n)
    s = s[np.argsort(-np.abs(s))]
    Rf = np.eye(n) - 2 * np.outer(u, u)
    S = Rf @ np.diag(s) @ Rf
    R, sb, d, err = P.shf(torch.tensor(S, device=dev()), 1, 30)
    torch.cuda.synchronize()
    assert float(err[-1]) < 1e-10 * np.linalg.norm(S) ** 2


def test_shf_no_reflectors():
    S = rand_sym(20, 5)
    R, sb, d, err = P.shf(torch.tensor(S, device=dev()), 0, 2)
    torch.cuda.synchronize()
    d = d.cpu().numpy()
    DSD = d[:, None] * S * d[None, :]
    off = DSD - np.diag(np.diag(DSD))
    assert np.allclose(sb.cpu().numpy(), np.diag(DSD))
    assert abs(float(err[-1]) - np.linalg.norm(off) ** 2) < 1e-10 * float(err[-1])
