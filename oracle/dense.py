"""Brute-force fixed point by a dense linear solve on tiny grids (test infrastructure only).

The sweep of ``oracle.sweep`` is the affine map f*' = T f* + g on the Q*n
post-collision state, with
    (T f*)_i(x) = (1 - omega) f*_i(x - v_i) + omega phi_i sum_j f*_j(x - v_j)
    g_i(x)      = chi_i S(x).
Its steady state solves (I - T) f* = g.  I - T is singular along the mass
mode, so the constraint sum_{i,x} f*_i(x) = 0 (the mass of the zero initial
state, conserved for a zero-mean source) is appended and the stacked system
is solved by least squares.  Phi is the post-stream moment sum_i f*_i(x - v_i).
"""
from __future__ import annotations

import numpy as np

from . import lattice as L
from .sweep import grid3


def _index(shape3, x, y, z):
    nx, ny, nz = shape3
    return ((z % nz) * ny + (y % ny)) * nx + (x % nx)


def fixed_point(lattice: str, order: int, tau_lb: float, s: np.ndarray):
    s = np.asarray(s, dtype=np.float64)
    lat = L.get(lattice)
    phi, chi = L.coefficients(lat, order)
    omega = 1.0 / tau_lb
    S = L.scaled_source(s, lat, tau_lb).reshape(-1)
    shape3 = grid3(s.shape)
    n = s.size
    Q = lat.Q
    v3 = lat.v3()
    T = np.zeros((Q * n, Q * n))
    for c in range(n):
        x = c % shape3[0]
        y = (c // shape3[0]) % shape3[1]
        z = c // (shape3[0] * shape3[1])
        src = [_index(shape3, x - v3[j, 0], y - v3[j, 1], z - v3[j, 2]) for j in range(Q)]
        for i in range(Q):
            row = i * n + c
            T[row, i * n + src[i]] += 1.0 - omega
            for j in range(Q):
                T[row, j * n + src[j]] += omega * phi[i]
    g = np.concatenate([chi[i] * S for i in range(Q)])
    M = np.vstack([np.eye(Q * n) - T, np.ones((1, Q * n))])
    rhs = np.concatenate([g, [0.0]])
    f, *_ = np.linalg.lstsq(M, rhs, rcond=None)
    f = f.reshape(Q, n)
    Phi = np.zeros(n)
    for c in range(n):
        x = c % shape3[0]
        y = (c // shape3[0]) % shape3[1]
        z = c // (shape3[0] * shape3[1])
        for j in range(Q):
            Phi[c] += f[j, _index(shape3, x - v3[j, 0], y - v3[j, 1], z - v3[j, 2])]
    return Phi.reshape(s.shape)
