"""Exact fixed point of the lattice iteration on a periodic grid (test infrastructure only).

The sweep of ``oracle.sweep`` is linear and shift-invariant, so each Fourier
mode k evolves on its own.  With E_i = exp(-i k.v_i) (streaming by v_i) and
a = 1 - omega, the fixed point of
    f*_i = a E_i f*_i + omega phi_i Phi + chi_i S,   Phi = sum_i E_i f*_i
is, with G_i = E_i / (1 - a E_i),
    Phi_hat (1 - omega sum_i phi_i G_i) = S_hat sum_i chi_i G_i.
For a lattice closed under v -> -v with even phi, chi, pairing i with -i and
using sum_i phi_i = 1 gives the cancellation-free real form (theta_i = k.v_i,
s_i = sin(theta_i / 2)):
    D(k) = sum_i phi_i 2 (2 - omega) s_i^2 / (omega^2 + 4 a s_i^2)
    A(k) = sum_i chi_i (cos theta_i - a)    / (omega^2 + 4 a s_i^2)
    Phi_hat(k) = S_hat(k) A(k) / D(k),  Phi_hat(0) = 0 (the initial mass).
Phi here is the post-stream moment, the quantity the sweep outputs.  The
phases k.v_i are reduced exactly in integer arithmetic before the sine and
cosine are taken.
"""
from __future__ import annotations

import numpy as np

from . import lattice as L


def _phase_index(shape, v):
    """Integer p with k.v = 2 pi p / prod(n) for every mode of the grid."""
    shape3 = tuple(shape)[::-1]        # (nx, ny, nz...) order of v components
    ntot = int(np.prod(shape3))
    p = np.zeros(tuple(shape), dtype=np.int64)
    for a, na in enumerate(shape3):
        m = np.arange(na, dtype=np.int64)
        # axis for component a is the (dim-1-a)-th array axis
        ax = len(shape3) - 1 - a
        bshape = [1] * len(shape3)
        bshape[ax] = na
        p = p + (m * int(v[a]) * (ntot // na)).reshape(bshape)
    p = np.mod(p, ntot)
    p = np.where(p > ntot // 2, p - ntot, p)   # theta in (-pi, pi]
    return p, ntot


def transfer(shape, lattice: str, order: int, tau_lb: float):
    """A(k)/D(k) for every mode of the grid (the k = 0 entry is set to 0)."""
    lat = L.get(lattice)
    phi, chi = L.coefficients(lat, order)
    omega = 1.0 / tau_lb
    a = 1.0 - omega
    A = np.zeros(tuple(shape))
    D = np.zeros(tuple(shape))
    for i, v in enumerate(lat.v):
        p, ntot = _phase_index(shape, v)
        theta = (2.0 * np.pi / ntot) * p
        s = np.sin(0.5 * theta)
        s2 = s * s
        den = omega * omega + 4.0 * a * s2
        A += chi[i] * (np.cos(theta) - a) / den
        D += phi[i] * 2.0 * (2.0 - omega) * s2 / den
    zero = (0,) * len(shape)
    R = np.zeros(tuple(shape))
    nz = D != 0.0
    R[nz] = A[nz] / D[nz]
    R[zero] = 0.0
    return R


def fixed_point(lattice: str, order: int, tau_lb: float, s: np.ndarray):
    """Steady-state Phi for Poisson right-hand side s (zero-mean) on its grid."""
    s = np.asarray(s, dtype=np.float64)
    lat = L.get(lattice)
    S = L.scaled_source(s, lat, tau_lb)
    R = transfer(s.shape, lattice, order, tau_lb)
    return np.real(np.fft.ifftn(np.fft.fftn(S) * R))


def transfer_c(shape, lattice: str, order: int, tau_lb: float, half: bool = False):
    """The same A(k)/D(k) from the plain C loop of ``spectral.c`` (OpenMP, one
    sine/cosine table over the grid's common phase denominator), for grids
    where the per-velocity numpy passes are slow.  half=True returns only the
    modes of a real FFT (last axis nx//2 + 1), which suffice since R is even."""
    from .sweep import _lib, grid3
    lat = L.get(lattice)
    phi, chi = L.coefficients(lat, order)
    nx, ny, nz = grid3(shape)
    nkx = nx // 2 + 1 if half else nx
    R = np.empty(tuple(shape)[:-1] + (nkx,))
    v3 = np.ascontiguousarray(lat.v3())
    rc = _lib().oracle_transfer(nx, ny, nz, nkx, lat.Q, v3.ctypes.data, 1.0 / float(tau_lb),
                                np.ascontiguousarray(phi).ctypes.data,
                                np.ascontiguousarray(chi).ctypes.data, R.ctypes.data)
    if rc:
        raise RuntimeError(f"oracle_transfer rejected its arguments ({rc})")
    return R


def fixed_point_large(lattice: str, order: int, tau_lb: float, s: np.ndarray, workers: int = -1):
    """``fixed_point`` for large grids: real FFTs (scipy, ``workers`` threads)
    and the half-spectrum transfer of ``transfer_c``.  Same formula."""
    import scipy.fft as F
    s = np.asarray(s, dtype=np.float64)
    lat = L.get(lattice)
    S = L.scaled_source(s, lat, tau_lb)
    Sh = F.rfftn(S, workers=workers)
    del S
    Sh *= transfer_c(s.shape, lattice, order, tau_lb, half=True)
    return F.irfftn(Sh, s=s.shape, workers=workers)


def continuum_poisson(s: np.ndarray):
    """Spectral solution of the continuum periodic Poisson problem lap(Phi) = -s."""
    s = np.asarray(s, dtype=np.float64)
    k2 = np.zeros(s.shape)
    for ax, n in enumerate(s.shape):
        k = 2.0 * np.pi * np.fft.fftfreq(n)
        bshape = [1] * s.ndim
        bshape[ax] = n
        k2 = k2 + (k ** 2).reshape(bshape)
    sh = np.fft.fftn(s)
    out = np.zeros_like(sh)
    nz = k2 > 0
    out[nz] = sh[nz] / k2[nz]
    return np.real(np.fft.ifftn(out))
