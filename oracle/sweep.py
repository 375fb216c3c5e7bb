"""Time-stepping oracle: the discrete lattice BGK iteration (test infrastructure only).

The paper never prints the discrete update; it is read here as the standard
lattice discretisation of Eq. (boltzmann) with time step 1 and the separable
equilibrium and source of Sec. 4:

    stream:   f_i(x)   = f*_i(x - v_i)                    (periodic)
    moment:   Phi(x)   = sum_i f_i(x)
    collide:  f*_i'(x) = (1 - omega) f_i(x) + omega phi_i Phi(x) + chi_i S(x)

with omega = 1/tau_lb and S = s c_s^2 (tau_lb - 1/2) (Sec. 5).  The answer of
the method is Phi at steady state.  Two implementations of the same sweep:
``sweep_c`` (plain C, OpenMP over cells, ``sweep.c``) and ``sweep_roll``
(numpy ``roll``, for cross-checking the C one on small grids).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import lattice as L

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        from .build import LIB, build
        build(force=False)      # compiles only when missing or older than its sources
        lib = ctypes.CDLL(LIB)
        lib.oracle_sweep.restype = ctypes.c_int
        lib.oracle_sweep.argtypes = [
            ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_transfer.restype = ctypes.c_int
        lib.oracle_transfer.argtypes = [
            ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _LIB = lib
    return _LIB


def threads() -> int:
    """OpenMP threads the C sweep uses."""
    return _lib().oracle_threads()


def grid3(shape):
    """(nx, ny, nz) of a field stored as (nz, ny, nx) / (ny, nx) / (nx,)."""
    s = tuple(shape)[::-1]
    return (s + (1, 1, 1))[:3]


class Problem:
    """One periodic Poisson problem for the oracle."""

    def __init__(self, lattice: str, order: int, tau_lb: float, s: np.ndarray, drift=None):
        self.lat = L.get(lattice)
        self.order = order
        self.tau_lb = float(tau_lb)
        self.omega = 1.0 / self.tau_lb
        if drift is None or not any(drift):
            self.phi, self.chi = L.coefficients(self.lat, order)
        else:  # advection-diffusion variant (oracle.drift)
            from . import drift as DR
            self.phi, self.chi = DR.coefficients(self.lat, order, drift)
        self.s = np.ascontiguousarray(s, dtype=np.float64)
        if self.s.ndim != self.lat.dim:
            raise ValueError("source rank must equal the lattice dimension")
        self.S = L.scaled_source(self.s, self.lat, self.tau_lb)
        self.shape = self.s.shape
        self.n = self.s.size
        self.v3 = np.ascontiguousarray(self.lat.v3())

    def zero_state(self):
        return np.zeros((self.lat.Q,) + self.shape)


def sweep_c(p: Problem, fin: np.ndarray, fout: np.ndarray, Phi: np.ndarray | None = None):
    """One sweep with the C oracle; fin -> fout, optional Phi output."""
    nx, ny, nz = grid3(p.shape)
    for a in (fin, fout) + ((Phi,) if Phi is not None else ()):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    assert fin.size == p.lat.Q * p.n and fout.size == p.lat.Q * p.n
    rc = _lib().oracle_sweep(
        nx, ny, nz, p.lat.Q, p.v3.ctypes.data, p.omega,
        p.phi.ctypes.data, p.chi.ctypes.data, p.S.ctypes.data,
        fin.ctypes.data, fout.ctypes.data,
        None if Phi is None else Phi.ctypes.data)
    if rc:
        raise RuntimeError("oracle_sweep rejected its arguments")


def sweep_roll(p: Problem, fin: np.ndarray):
    """One sweep with numpy roll; returns (fout, Phi)."""
    axes = tuple(range(-1, -p.lat.dim - 1, -1))   # x, y, z -> last axes
    f = np.empty_like(fin)
    for i, v in enumerate(p.lat.v):
        f[i] = np.roll(fin[i], shift=tuple(int(c) for c in v), axis=axes)
    Phi = np.zeros(p.shape)
    for i in range(p.lat.Q):
        Phi = Phi + f[i]
    fout = np.empty_like(fin)
    for i in range(p.lat.Q):
        fout[i] = (1.0 - p.omega) * f[i] + p.omega * p.phi[i] * Phi + p.chi[i] * p.S
    return fout, Phi


def run(p: Problem, sweeps: int, f0: np.ndarray | None = None):
    """Run a fixed number of sweeps from f0 (default 0); returns (Phi, f*)."""
    a = p.zero_state() if f0 is None else np.array(f0, dtype=np.float64, copy=True)
    b = np.empty_like(a)
    Phi = np.zeros(p.shape)
    for _ in range(sweeps):
        sweep_c(p, a, b, Phi)
        a, b = b, a
    return Phi, a


def solve_maxchange(p: Problem, tol: float, max_sweeps: int):
    """Sweep from f* = 0 until max_x |Phi_t - Phi_{t-1}| < tol.

    Every sweep is counted, the first one included; the change is defined from
    the second sweep on.  Returns (Phi, sweeps, last max change).
    """
    a = p.zero_state()
    b = np.empty_like(a)
    Phi = np.zeros(p.shape)
    prev = np.zeros(p.shape)
    change = np.inf
    for t in range(1, max_sweeps + 1):
        sweep_c(p, a, b, Phi)
        a, b = b, a
        if t >= 2:
            change = float(np.max(np.abs(Phi - prev)))
            if change < tol:
                return Phi.copy(), t, change
        prev, Phi = Phi, prev
        Phi[...] = 0.0
    raise RuntimeError(f"no convergence in {max_sweeps} sweeps (change {change})")
