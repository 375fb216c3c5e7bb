"""Advection-diffusion variant of the scheme (test infrastructure only).

The paper names time-dependent diffusion and advection-diffusion as the next
extensions of the method (Sec. 6) and fixes no scheme for them.  Reading used
here: the sweep is unchanged, and the equilibrium shape phi_i Phi becomes that
of a Gaussian moved by a uniform drift u.  The ratio of the moved to the
unmoved Gaussian at velocity v is exp(v.u / c^2 - |u|^2 / (2 c^2)); kept to
second order in u it adds

    w_i ( a_i + a_i^2 / 2 - b ),   a_i = v_i.u / c^2,   b = |u|^2 / (2 c^2)

to phi_i, while chi_i is unchanged.  The sweep is then a time step of
    d_t Phi + u . grad Phi = D lap Phi + D s,   D = c^2 (tau_lb - 1/2),
and its fixed point solves lap Phi - (u / D) . grad Phi = -s.

``transfer`` is the exact fixed point per Fourier mode, in the general
complex form (no symmetry of phi_i is assumed):
    Phi_hat (1 - omega sum_i phi_i G_i) = S_hat sum_i chi_i G_i,
    G_i = E_i / (1 - (1 - omega) E_i),  E_i = exp(-i k.v_i).
"""
from __future__ import annotations

import mpmath as mp
import numpy as np

from . import lattice as L
from . import spectral as SP


def coefficients_mp(lat: L.Lattice, order: int, u):
    """phi_i(u), chi_i (mpf lists) for drift u = (ux, uy, uz)."""
    phi, chi = L.coefficients_mp(lat, order)
    with mp.workdps(L.DPS):
        uu = [mp.mpf(float(x)) for x in tuple(u) + (0.0,) * (3 - len(tuple(u)))]
        c2 = lat.c2_mp
        b = mp.fsum(x * x for x in uu) / (2 * c2)
        out = []
        for vi, wi, p in zip(lat.v3(), lat.w_mp, phi):
            a = mp.fsum(mp.mpf(int(vi[k])) * uu[k] for k in range(3)) / c2
            out.append(p + wi * (a + a * a / 2 - b))
    return out, chi


def coefficients(lat: L.Lattice, order: int, u):
    phi, chi = coefficients_mp(lat, order, u)
    return np.array([float(x) for x in phi]), np.array([float(x) for x in chi])


def transfer(shape, lattice: str, order: int, tau_lb: float, u):
    """Complex Phi_hat / S_hat for every mode of the grid (0 at k = 0)."""
    lat = L.get(lattice)
    phi, chi = coefficients(lat, order, u)
    omega = 1.0 / tau_lb
    a = 1.0 - omega
    sp = np.zeros(tuple(shape), dtype=complex)
    sc = np.zeros(tuple(shape), dtype=complex)
    for i, v in enumerate(lat.v):
        p, ntot = SP._phase_index(shape, v)
        E = np.exp(-1j * (2.0 * np.pi / ntot) * p)
        G = E / (1.0 - a * E)
        sp += phi[i] * G
        sc += chi[i] * G
    den = 1.0 - omega * sp
    R = np.zeros(tuple(shape), dtype=complex)
    zero = (0,) * len(shape)
    nz = np.abs(den) > 0
    R[nz] = sc[nz] / den[nz]
    R[zero] = 0.0
    return R


def fixed_point(lattice: str, order: int, tau_lb: float, s: np.ndarray, u):
    """Steady Phi of the drifted scheme for right-hand side s (zero mean)."""
    s = np.asarray(s, dtype=np.float64)
    lat = L.get(lattice)
    S = L.scaled_source(s, lat, tau_lb)
    return np.real(np.fft.ifftn(np.fft.fftn(S) * transfer(s.shape, lattice, order, tau_lb, u)))


def continuum_mode(k, u, D):
    """Phi_hat / s_hat of lap Phi - (u / D) . grad Phi = -s for the mode exp(i k.x)."""
    k = np.asarray(k, dtype=float)
    u = np.asarray(u, dtype=float)[: len(k)]
    return 1.0 / (k @ k + 1j * (u @ k) / D)
