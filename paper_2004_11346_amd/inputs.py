"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the transform: it only knows the coefficient
layout (which degree k and order m sit in which slot) and draws random numbers.
All draws use ``numpy.random.Generator(PCG64(seed))`` in FP64; FP32 runs cast
the same draw.

Coefficient layout (m-major, complex): orders in the sequence
0, 1, -1, 2, -2, ..., 2N-1, -(2N-1); inside each order the degrees
k = |m| .. 2N-1.  There are exactly 4N^2 slots per field.

Grid layout: [2N rows][M = 4N-1 columns], row l = l-th Gauss-Legendre node in
ascending x = cos(theta), column j = phi_j = 2 pi (j + 1/2) / M.
"""
from __future__ import annotations

import numpy as np


def n_coefs(N: int) -> int:
    return 4 * N * N


def grid_shape(N: int):
    return (2 * N, 4 * N - 1)


def layout(N: int):
    """Return (k_of_slot, m_of_slot) int arrays of length 4N^2."""
    ks, ms = [], []
    n = 2 * N
    for a in range(n):
        for m in ((0,) if a == 0 else (a, -a)):
            ks.append(np.arange(a, n, dtype=np.int64))
            ms.append(np.full(n - a, m, dtype=np.int64))
    return np.concatenate(ks), np.concatenate(ms)


def slot(N: int, k: int, m: int) -> int:
    """Slot index of (k, m) in the m-major layout (by enumeration)."""
    a = abs(m)
    assert 0 <= a <= k < 2 * N
    off = 0
    for b in range(a):
        off += (2 * N - b) * (1 if b == 0 else 2)
    if m < 0:
        off += 2 * N - a
    return off + (k - a)


def config_seed(config: int, field: int) -> int:
    """Field ``field`` of workload ``config`` uses seed 1000*config + field."""
    return 1000 * config + field


def make_beta(N: int, batch: int, config: int, dist: str = "half") -> np.ndarray:
    """Complex coefficients [batch, 4N^2] (complex128).

    dist="half":  Re, Im iid N(0, 1/2)            (unit complex variance)
    dist="decay": beta = (a + i b) / (sqrt(2) (k + 1)), a, b iid N(0, 1)
                  (complex variance (k + 1)^-2)
    """
    out = np.empty((batch, n_coefs(N)), dtype=np.complex128)
    k_of = None
    if dist == "decay":
        k_of, _ = layout(N)
    for b in range(batch):
        rng = np.random.Generator(np.random.PCG64(config_seed(config, b)))
        re = rng.standard_normal(n_coefs(N))
        im = rng.standard_normal(n_coefs(N))
        if dist == "half":
            out[b] = (re + 1j * im) * np.sqrt(0.5)
        elif dist == "decay":
            out[b] = (re + 1j * im) / (np.sqrt(2.0) * (k_of + 1.0))
        else:
            raise ValueError(dist)
    return out


def make_grid(N: int, batch: int, config: int) -> np.ndarray:
    """Complex grid values [batch, 2N, M], Re and Im iid N(0, 1/2)."""
    out = np.empty((batch,) + grid_shape(N), dtype=np.complex128)
    for b in range(batch):
        rng = np.random.Generator(np.random.PCG64(config_seed(config, b) + 500))
        shp = grid_shape(N)
        out[b] = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) * np.sqrt(0.5)
    return out


def uneven_batch(seed: int = 4000, count: int = 64, sizes=(128, 256, 512, 1024)):
    """List of (N_t, fields_t) for the uneven persistent batch: N uniform over
    ``sizes``, fields uniform over 1..4."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ns = rng.choice(np.asarray(sizes), size=count)
    fs = rng.integers(1, 5, size=count)
    return [(int(a), int(b)) for a, b in zip(Ns, fs)]


def sample_indices(n: int, count: int, seed: int) -> np.ndarray:
    """Seeded sample of ``count`` distinct indices in [0, n), sorted."""
    rng = np.random.Generator(np.random.PCG64(seed))
    count = min(count, n)
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)
