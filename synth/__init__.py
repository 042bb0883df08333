"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module draws random numbers and nothing else: it holds none of the
method's arithmetic and imports neither the oracle nor the HIP package.  The
same generated tensor is handed to both sides of every comparison.

Two back ends:
  * numpy PCG64 (host), one independent stream per (seed, stream id), used for
    everything the CPU can generate quickly;
  * torch's device generator (Philox) for the multi-GiB benchmark batches,
    seeded from (seed, stream id); the values differ from the host back end,
    but each run generates a tensor once and gives the very same bits to the
    GPU path and to the oracle (copied back to the host).

Distributions follow the workloads of the paper's experiments as stated in the
benchmark configurations: Gaussian reflector vectors normalised to unit length,
Gaussian data, eigenvalues uniform on [0.1, 10] or log-uniform on [1e-2, 1e2].
"""
from __future__ import annotations

import numpy as np

# Stream ids: one per tensor role, so adding a tensor never shifts another.
STREAM_U, STREAM_LAM, STREAM_X, STREAM_XB, STREAM_W, STREAM_G = 1, 2, 3, 4, 5, 6


def host_rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream])))


def reflectors(n: int, h: int, seed: int = 0, normalize: bool = True) -> np.ndarray:
    """(h, n) float64; row k ~ N(0, I_n), optionally scaled to unit length."""
    U = host_rng(seed, STREAM_U).standard_normal((h, n))
    if normalize and h > 0:
        U = U / np.linalg.norm(U, axis=1, keepdims=True)
    return U


def structured_reflectors(n: int, h: int, seed: int = 0) -> np.ndarray:
    """(h, n) float64 with the sparsity of Householder QR reflectors (the
    remark after Result 3): row k (0-based) has k leading zeros, the rest
    N(0, 1), scaled to unit length."""
    U = host_rng(seed, STREAM_U).standard_normal((h, n))
    for k in range(min(h, n)):
        U[k, :k] = 0.0
    if h > 0:
        U = U / np.linalg.norm(U, axis=1, keepdims=True)
    return U


def eig_uniform(n: int, lo: float = 0.1, hi: float = 10.0, seed: int = 0) -> np.ndarray:
    return host_rng(seed, STREAM_LAM).uniform(lo, hi, size=n)


def eig_loguniform(n: int, lo_exp: float = -2.0, hi_exp: float = 2.0, seed: int = 0) -> np.ndarray:
    return 10.0 ** host_rng(seed, STREAM_LAM).uniform(lo_exp, hi_exp, size=n)


def gaussian(shape, seed: int = 0, stream: int = STREAM_X) -> np.ndarray:
    """float64 N(0, 1) on the host."""
    return host_rng(seed, stream).standard_normal(shape)


def device_gaussian(shape, seed: int = 0, stream: int = STREAM_X, device="cuda",
                    dtype=None):
    """N(0, 1) drawn directly in device memory by torch's generator, in float32,
    then cast (round to nearest even) to ``dtype`` if given."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed((int(seed) * 1_000_003 + int(stream) * 7919) & 0x7FFFFFFFFFFFFFFF)
    x = torch.randn(shape, generator=g, device=device, dtype=torch.float32)
    if dtype is not None and dtype != torch.float32:
        x = x.to(dtype)
    return x
