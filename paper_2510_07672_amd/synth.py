"""Seeded synthetic initial conditions.

Holds no arithmetic of the method: only the random or closed-form
starting fields that the GPU path, the oracle, the tests and the
benchmark are all handed.  Every generator returns float64 numpy arrays
shaped [B, N, N] (C-contiguous, u[b, i, j] = u(x_i, y_j)).
"""

from __future__ import annotations

import numpy as np


def random_ic(n: int, seeds, amp: float = 0.9) -> np.ndarray:
    """i.i.d. uniform(-amp, amp) per grid point, one field per seed.

    Stand-in for the random grain-coarsening start of Section 4.2 (read as
    uniform on (-0.9, 0.9) so that both phases are present).
    """
    seeds = [int(s) for s in np.atleast_1d(seeds)]
    out = np.empty((len(seeds), n, n), dtype=np.float64)
    for b, s in enumerate(seeds):
        out[b] = np.random.default_rng(s).uniform(-amp, amp, size=(n, n))
    return out


def bubbles_ic(n: int, eps: float, length: float = 1.0) -> np.ndarray:
    """Two merging bubbles (the closed-form start of Section 4.2.1).

    The paper's domain [-0.5, 0.5]^2 is shifted to [0, L)^2 by +L/2.
    """
    h = length / n
    x = np.arange(n) * h - 0.5 * length
    X, Y = np.meshgrid(x, x, indexing="ij")
    r1 = np.sqrt((X - 0.14) ** 2 + Y ** 2)
    r2 = np.sqrt((X + 0.14) ** 2 + Y ** 2)
    u = np.maximum(np.tanh((0.2 - r1) / eps), np.tanh((0.2 - r2) / eps))
    return u[None].astype(np.float64)


def single_mode(n: int, kx: int, ky: int, amp: float) -> np.ndarray:
    """amp * cos(2 pi (kx i + ky j) / n) on the n x n grid, shape [1, n, n]."""
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    return (amp * np.cos(2.0 * np.pi * (kx * i + ky * j) / n))[None].astype(np.float64)
