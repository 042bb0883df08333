"""k nearest neighbours in the learned metric (Sec. IV-C): P.knn transforms
queries and database by L = diag(sqrt(lam)) Q^T on the fused kernels, then
hh_knn ranks all pairs.  The oracle computes every pair's distance by the
definition d(x, y) = sum_i lam_i ((Q^T (x - y))_i)^2 (oracle.mahal, FP64) and
sorts each row (stable).

What is unique is compared exactly: the k smallest distances of each query
(sorted), and the index set wherever the k-th distance is separated from the
next by more than the tolerance.  Tolerance: candidates are ranked by the
expanded form ||a||^2 + ||b||^2 - 2 a^T b in FP32, whose error is a few units
of rounding of ||a||^2 + ||b||^2, so returned distances are checked to
1e-5 (||z_q||^2 + the largest ||z_j||^2 among the neighbours), and every
returned index must carry the distance returned for it (recomputed from the
differences) to the same tolerance.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1811_07624_amd")


def dev():
    return torch.device("cuda:0")


def case(n, h, Nq, Nd, seed, dup=0):
    U = synth.reflectors(n, h, seed=seed)
    lam = synth.eig_uniform(n, seed=seed)
    Xq = synth.gaussian((Nq, n), seed=seed, stream=synth.STREAM_X)
    Xd = synth.gaussian((Nd, n), seed=seed, stream=synth.STREAM_XB)
    if dup:
        Xd[dup:2 * dup] = Xd[:dup]  # repeated database rows: equal distances
    f = lambda a: np.asarray(a, np.float32).astype(np.float64)  # the bits the GPU sees
    return f(U), f(lam), f(Xq), f(Xd)


def oracle_dist(U, lam, Xq, Xd):
    Nq, Nd = Xq.shape[0], Xd.shape[0]
    A = np.repeat(Xq, Nd, axis=0)
    B = np.tile(Xd, (Nq, 1))
    return oracle.mahal(U, lam, A, B).reshape(Nq, Nd)


@pytest.mark.parametrize("n,h,Nq,Nd,k,dup", [(40, 6, 100, 1500, 5, 0), (100, 7, 70, 777, 10, 0),
                                             (200, 8, 65, 64, 32, 0), (3, 2, 5, 40, 1, 0),
                                             (64, 6, 130, 300, 8, 20), (224, 8, 33, 129, 4, 0)])
def test_knn_matches_oracle(n, h, Nq, Nd, k, dup):
    U, lam, Xq, Xd = case(n, h, Nq, Nd, seed=n + Nd, dup=dup)
    t = lambda a: torch.tensor(a, dtype=torch.float32, device=dev())
    d, idx = P.knn(t(U), t(lam), t(Xq), t(Xd), k)
    sq = torch.sqrt(t(lam))
    Zq = P.signed_raw("apply_T", t(U), t(Xq), d_out=sq).double().cpu().numpy()
    Zd = P.signed_raw("apply_T", t(U), t(Xd), d_out=sq).double().cpu().numpy()
    torch.cuda.synchronize()
    d, idx = d.double().cpu().numpy(), idx.cpu().numpy()
    D = oracle_dist(U, lam, Xq, Xd)
    order = np.argsort(D, axis=1, kind="stable")
    ref = np.take_along_axis(D, order, axis=1)
    for q in range(Nq):
        assert len(set(idx[q])) == k and idx[q].min() >= 0 and idx[q].max() < Nd
        assert (np.diff(d[q]) >= 0).all()
        scale = (Zq[q] ** 2).sum() + (Zd[idx[q]] ** 2).sum(axis=1).max()
        tol = 1e-5 * scale
        assert np.abs(d[q] - ref[q, :k]).max() <= tol, q
        assert np.abs(D[q, idx[q]] - d[q]).max() <= tol, q
        if k < Nd and ref[q, k] - ref[q, k - 1] > 2 * tol:
            assert set(idx[q]) == set(order[q, :k]), q
    if dup:  # equal distances keep the smaller index first
        for q in range(Nq):
            for j in range(k - 1):
                if d[q, j] == d[q, j + 1]:
                    assert idx[q, j] < idx[q, j + 1]


def test_knn_empty_queries():
    Z = torch.randn((10, 8), device=dev())
    d, idx = P.knn_raw(Z[:0], Z, 3)
    assert d.shape == (0, 3) and idx.shape == (0, 3)
