"""Seeded synthetic Poisson right-hand sides (inputs only, no solver arithmetic).

Shared by the tests, the benchmark and the oracle checks so that the GPU path
and the CPU oracle see identical inputs.  Fields are FP64, stored with x
fastest: shape (nx,), (ny, nx) or (nz, ny, nx).
"""
from __future__ import annotations

import numpy as np


def sine_product(shape, modes=None) -> np.ndarray:
    """prod_a sin(2 pi m_a x_a / n_a) on integer cells (default m_a = 1)."""
    shape = tuple(shape)
    modes = modes or (1,) * len(shape)
    out = np.ones(shape)
    for ax, (n, m) in enumerate(zip(shape, modes)):
        x = np.arange(n)
        b = [1] * len(shape)
        b[ax] = n
        out = out * np.sin(2 * np.pi * m * x / n).reshape(b)
    return out


def gaussian_blobs(shape, count: int, sigma: float, seed: int, amplitudes: str = "normal",
                   radius_sigmas: float = 8.0) -> np.ndarray:
    """Sum of `count` periodic Gaussians exp(-r^2 / (2 sigma^2)).

    Centres are uniform on [0, n_a) per axis (continuous), distances use the
    periodic minimum image, and each blob is evaluated within radius_sigmas *
    sigma of its centre (the tail beyond is below exp(-32)).  Amplitudes:
    "normal" ~ N(0, 1); "signed_uniform" ~ +-U(1, 10) with a fair random sign.
    The draw order is centres (count x dim), then amplitudes (and signs).
    """
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(count, d)) * np.array(shape[::-1], dtype=np.float64)
    if amplitudes == "normal":
        amp = rng.standard_normal(count)
    elif amplitudes == "signed_uniform":
        mag = rng.uniform(1.0, 10.0, size=count)
        sign = np.where(rng.integers(0, 2, size=count) == 1, 1.0, -1.0)
        amp = sign * mag
    else:
        raise ValueError(amplitudes)
    out = np.zeros(shape)
    R = int(np.ceil(radius_sigmas * sigma))
    off = np.arange(-R, R + 1)
    inv = 1.0 / (2.0 * sigma * sigma)
    for c, a in zip(centres, amp):
        # per axis (x first in c): nearest cell, local offsets, 1D factors
        idx, fac = [], []
        for ax in range(d):
            n = shape[::-1][ax]
            base = int(np.floor(c[ax]))
            cells = base + off
            dist = cells - c[ax]
            dist = dist - n * np.round(dist / n)
            keep = np.abs(dist) <= radius_sigmas * sigma
            cells, dist = cells[keep], dist[keep]
            idx.append(np.mod(cells, n))
            fac.append(np.exp(-dist * dist * inv))
        if d == 1:
            np.add.at(out, idx[0], a * fac[0])
        elif d == 2:
            blk = a * np.outer(fac[1], fac[0])
            np.add.at(out, np.ix_(idx[1], idx[0]), blk)
        else:
            blk = a * fac[2][:, None, None] * fac[1][None, :, None] * fac[0][None, None, :]
            np.add.at(out, np.ix_(idx[2], idx[1], idx[0]), blk)
    return out


def zero_mean(s: np.ndarray) -> np.ndarray:
    return s - s.mean()


def poisson_source(kind: str, shape, seed: int = 12345) -> np.ndarray:
    """Named source recipes of the benchmark configurations (zero-mean FP64)."""
    shape = tuple(shape)
    if kind == "sine":
        return sine_product(shape)
    if kind == "blobs2d":        # 64 Gaussians, width 2 cells, N(0,1) amplitudes
        return zero_mean(gaussian_blobs(shape, 64, 2.0, seed))
    if kind == "blobs3d":        # 512 Gaussians, width 1.5 cells, N(0,1) + sine background
        s = gaussian_blobs(shape, 512, 1.5, seed) + sine_product(shape)
        return zero_mean(s)
    if kind == "stiff3d":        # 4096 point-like Gaussians, width 1, +-U(1,10)
        return zero_mean(gaussian_blobs(shape, 4096, 1.0, seed, "signed_uniform"))
    if kind == "noise":
        rng = np.random.default_rng(seed)
        return zero_mean(rng.standard_normal(shape))
    raise ValueError(kind)
