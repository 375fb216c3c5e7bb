"""Pins of the oracle's Knudsen mapping and stability analysis against
measurements of the oracle's own time stepping (CPU).

* The Knudsen number (Sec. 2: Kn = lambda / L, with the diffusivity
  D = c_s^2 tau) is checked through a measured diffusivity: a single Fourier
  mode's decay under the time-stepped scheme gives D, hence the mean free path
  lambda = c_s tau = D / c_s, and lambda / L must give back the Kn that
  ``lattice.tau_from_knudsen`` was asked for.
* The von Neumann amplification (``generator.max_amplification``) is checked
  against the per-sweep growth of random populations under the time-stepped
  scheme on a grid whose modes are exactly the analysed wavevectors.
* The product's stability limits (read through the C ABI on the host) are
  shown stable by that analysis on the library's sets.
"""
import ctypes

import numpy as np
import pytest

from oracle import generator as G
from oracle import lattice as L
from oracle import sweep as SW


def _decay_diffusivity(lattice, order, tau, shape, t1=200, t2=800):
    """D from the decay of Phi0 = cos(2 pi x / nx) started at its equilibrium
    f*_i = phi_i Phi0 with no source: the amplitude falls by exp(-D k^2) per
    sweep once the non-hydrodynamic modes (factor 1 - omega) have died out."""
    lat = L.get(lattice)
    p = SW.Problem(lattice, order, tau, np.zeros(shape))
    nx = shape[-1]
    k = 2.0 * np.pi / nx
    phi0 = np.broadcast_to(np.cos(k * np.arange(nx)), shape).copy()
    cphi, _ = L.coefficients(lat, order)
    f0 = cphi.reshape((-1,) + (1,) * len(shape)) * phi0[None]
    P1, f1 = SW.run(p, t1, f0)
    P2, _ = SW.run(p, t2 - t1, f1)
    a1, a2 = float(np.sum(P1 * phi0)), float(np.sum(P2 * phi0))
    return -np.log(a2 / a1) / (k * k * (t2 - t1))


CASES_KN = [("D1Q5", 3, 0.01, (256,)), ("D1Q9", 5, 0.01, (256,)), ("D1Q13", 7, 0.01, (256,)),
            ("D2Q25", 1, 0.01, (64, 128)), ("D2Q81", 5, 0.01, (64, 128))]


@pytest.mark.parametrize("lattice,order,kn,shape", CASES_KN)
def test_knudsen_mapping_from_measured_diffusivity(lattice, order, kn, shape):
    """tau_from_knudsen(Kn) -> time-stepped decay -> D -> lambda = D / c_s ->
    lambda / L with L the smallest box side: Kn comes back within 2 %
    (the diffusive limit holds to O((k lambda)^2), k lambda ~ 0.03-0.06 here).
    The 2D boxes are 64 x 128 with the mode along the long side, so a mapping
    that took the longest side would be a factor 2 off."""
    lat = L.get(lattice)
    box = min(shape)
    tau = L.tau_from_knudsen(kn, lat, box)
    D = _decay_diffusivity(lattice, order, tau, shape)
    cs = float(np.sqrt(lat.c2))
    assert abs(D / (lat.c2 * (tau - 0.5)) - 1) < 0.02       # D = c_s^2 (tau_lb - 1/2)
    assert abs((D / cs) / box / kn - 1) < 0.02              # Kn = lambda / L


@pytest.mark.parametrize("planted", ["cs2_for_cs", "tau_lb_for_tau", "longest_side"])
def test_knudsen_mapping_rejects_planted_readings(planted):
    """Plausible misreadings of the mapping move the measured Kn by > 5 %."""
    lattice, order, kn, shape = "D2Q81", 5, 0.01, (64, 128)
    lat = L.get(lattice)
    cs = float(np.sqrt(lat.c2))
    if planted == "cs2_for_cs":
        tau = 0.5 + kn * 64 / lat.c2
    elif planted == "tau_lb_for_tau":
        tau = kn * 64 / cs
    else:
        tau = L.tau_from_knudsen(kn, lat, 128)
    D = _decay_diffusivity(lattice, order, tau, shape)
    assert abs((D / cs) / 64 / kn - 1) > 0.05


def _growth(lattice, order, tau, shape, t1=200, t2=500):
    """Per-sweep growth of ||f*|| from random populations, no source."""
    lat = L.get(lattice)
    p = SW.Problem(lattice, order, tau, np.zeros(shape))
    f0 = np.random.default_rng(0).standard_normal((lat.Q,) + shape)
    _, f1 = SW.run(p, t1, f0)
    _, f2 = SW.run(p, t2 - t1, f1)
    return (np.linalg.norm(f2) / np.linalg.norm(f1)) ** (1.0 / (t2 - t1))


@pytest.mark.parametrize("lattice,order,tau,shape,t1,t2", [
    ("D2Q81", 5, 0.55, (8, 8), 200, 500), ("D2Q169", 7, 0.7, (8, 8), 200, 500),
    ("D3Q111", 5, 0.6, (8, 8, 8), 200, 500), ("D1Q13", 7, 0.7, (64,), 1000, 3000),
    ("D1Q9", 5, 0.6, (64,), 1000, 3000)])
def test_amplification_equals_time_stepped_growth(lattice, order, tau, shape, t1, t2):
    """Below the stability limit the largest amplification over the grid's
    wavevectors (nk = the grid's side) is the growth rate the time-stepped
    scheme shows on that grid, to 1e-9 (the window starts once the other
    modes have fallen behind the fastest-growing one)."""
    r = G.lattice_spectral_radius(lattice, order, tau, nk=shape[0])
    g = _growth(lattice, order, tau, shape, t1, t2)
    assert r > 1.001
    assert abs(g / r - 1) < 1e-9


def _lib():
    from paper_1504_05869_amd import _lib as PL
    return PL


def _accepted(lattice, order, tau):
    """Whether the product's lkp_create validation accepts tau_lb (host only:
    lkp_footprint_bytes returns 0 for a description it rejects)."""
    PL = _lib()
    lib = PL.load()
    info_dim = L.get(lattice).dim
    d = PL.ProblemDesc()
    d.dim = info_dim
    for a in range(3):
        d.n[a] = 16 if a < info_dim else 1
    d.lattice = PL.LATTICES[lattice]
    d.order = order
    d.precision = 0
    d.tau_lb = tau
    return lib.lkp_footprint_bytes(ctypes.byref(d)) > 0


@pytest.mark.parametrize("lattice,order", [("D2Q81", 5), ("D2Q37", 5), ("D3Q111", 5), ("D3Q107", 5),
                                           ("D2Q169", 7), ("D2Q77", 7), ("D1Q9", 5),
                                           ("D1Q13", 7)])
def test_product_stability_limits_are_stable(lattice, order):
    """The smallest tau_lb the library accepts (found by bisection through the
    C ABI) gives no growing mode on the library's set, nor do larger tau_lb up
    to the 512^3 workload's 184.36; and the scheme does grow somewhere below
    that limit (the limit is not vacuous)."""
    lo, hi = 0.5, 2.0
    assert _accepted(lattice, order, hi) and not _accepted(lattice, order, 0.5)
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        lo, hi = (lo, mid) if _accepted(lattice, order, mid) else (mid, hi)
    limit = hi
    nk = {1: 64, 2: 16, 3: 8}[L.get(lattice).dim]
    for tau in (limit, 1.0, 184.36):
        assert G.lattice_spectral_radius(lattice, order, tau, nk) <= 1 + 1e-12, tau
    below = [G.lattice_spectral_radius(lattice, order, t, nk) for t in (0.52, 0.55, 0.6, 0.7)
             if t < limit]
    assert max(below) > 1.001
