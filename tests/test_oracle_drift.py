"""Pins of the advection-diffusion oracle (oracle/drift.py) against what the
mathematics fixes: the drifted Gaussian's moments, the u = 0 special case,
the closed-form steady mode of lap Phi - (u/D).grad Phi = -s, the transient
decay and phase speed of a mode, and a planted sign mistake."""
import mpmath as mp
import numpy as np
import pytest

from oracle import drift as DR
from oracle import lattice as L
from oracle import spectral as SP
from oracle import sweep as SW

SETS = [("D1Q9", 5), ("D2Q9", 3), ("D2Q81", 5), ("D2Q37", 5), ("D2Q169", 7), ("D3Q111", 5)]


def _u(dim):
    return (0.05, -0.03, 0.02)[:dim]


@pytest.mark.parametrize("name,order", SETS)
def test_zero_drift_is_the_diffusion_scheme(name, order):
    lat = L.get(name)
    phi0, chi0 = L.coefficients_mp(lat, order)
    phi, chi = DR.coefficients_mp(lat, order, (0.0, 0.0, 0.0))
    assert all(a == b for a, b in zip(phi, phi0)) and all(a == b for a, b in zip(chi, chi0))


@pytest.mark.parametrize("name,order", SETS)
def test_drifted_equilibrium_has_the_moved_gaussian_moments(name, order):
    """sum phi_i = 1, sum phi_i v_i = u, sum phi_i v_i v_j = c^2 delta + u u
    (50-digit arithmetic): mass, drift and the moved second moment."""
    lat = L.get(name)
    u = _u(lat.dim)
    phi, _ = DR.coefficients_mp(lat, order, u)
    V = lat.v3()
    with mp.workdps(L.DPS):
        tol = mp.mpf(10) ** -40
        uu = [mp.mpf(float(x)) for x in u] + [mp.mpf(0)] * (3 - lat.dim)
        assert abs(mp.fsum(phi) - 1) < tol
        for a in range(lat.dim):
            m1 = mp.fsum(p * int(v[a]) for p, v in zip(phi, V))
            assert abs(m1 - uu[a]) < tol
            for b in range(lat.dim):
                m2 = mp.fsum(p * int(v[a]) * int(v[b]) for p, v in zip(phi, V))
                want = (lat.c2_mp if a == b else 0) + uu[a] * uu[b]
                assert abs(m2 - want) < tol


def _mode_error(name, order, tau, n, u, u_cont=None):
    """Relative distance of the scheme's steady response to the mode k = 2 pi / n
    along x from the continuum one (u_cont: drift used for the continuum)."""
    lat = L.get(name)
    shape = (1,) * (lat.dim - 1) + (n,)
    R = DR.transfer(shape, name, order, tau, u)
    D = lat.c2 * (tau - 0.5)
    disc = R[(0,) * (lat.dim - 1) + (1,)] * D
    k = (2 * np.pi / n,) + (0.0,) * (lat.dim - 1)
    cont = DR.continuum_mode(k, u if u_cont is None else u_cont, D)
    return abs(disc - cont) / abs(cont)


@pytest.mark.parametrize("name,order", SETS[1:])
@pytest.mark.parametrize("tau", [1.0, 2.0])
def test_steady_mode_converges_to_closed_form(name, order, tau):
    """Phi_hat / s_hat -> 1 / (k^2 + i u.k / D) as k -> 0, at first order in k
    or better (the drift terms are exact to second moments only)."""
    u = _u(L.get(name).dim)
    e = [_mode_error(name, order, tau, n, u) for n in (32, 64, 128, 256)]
    assert e[-1] < 5e-3
    assert e[0] / e[-1] > 8.0
    assert all(b < a for a, b in zip(e, e[1:]))


def test_planted_sign_mistake_fails_closed_form():
    """Drifting against u gives an O(1) error that does not shrink with k."""
    u = (0.05, -0.03)
    for n in (64, 256):
        assert _mode_error("D2Q81", 5, 1.0, n, tuple(-x for x in u), u_cont=u) > 0.5


def test_transient_mode_decays_and_travels_at_the_continuum_rate():
    """Time-dependent use: from f*_i = phi_i(u) cos(k x) with no source, the
    mode's amplitude changes per sweep by exp(-(i u.k + D k^2)) to O(k)."""
    name, order, tau, n, u = "D2Q81", 5, 1.0, 64, (0.05, 0.03)
    lat = L.get(name)
    D, k = lat.c2 * (tau - 0.5), 2 * np.pi / n
    x = np.arange(n)
    phi0 = np.tile(np.cos(k * x), (n, 1))
    p = SW.Problem(name, order, tau, np.zeros((n, n)), drift=u)
    f = p.phi[:, None, None] * phi0[None]
    b, Phi = np.empty_like(f), np.empty((n, n))
    amp = {}
    for t in range(1, 301):
        SW.sweep_c(p, f, b, Phi)
        f, b = b, f
        if t in (100, 300):
            amp[t] = np.fft.fft2(Phi)[0, 1]
    lam = np.log(amp[300] / amp[100]) / 200
    want = -(1j * u[0] * k + D * k * k)
    assert abs(lam - want) / abs(want) < 5e-3


def test_sweep_fixed_point_equals_spectral():
    """The C oracle's sweep, iterated to convergence with a drift, reaches the
    complex spectral fixed point (two independent computations)."""
    name, order, tau, u = "D2Q81", 5, 1.7, (0.1, -0.07)
    rng = np.random.default_rng(3)
    s = rng.standard_normal((12, 10))
    s -= s.mean()
    p = SW.Problem(name, order, tau, s, drift=u)
    f, b, Phi = p.zero_state(), p.zero_state(), np.empty(s.shape)
    for _ in range(6000):
        SW.sweep_c(p, f, b, Phi)
        f, b = b, f
    ref = DR.fixed_point(name, order, tau, s, u)
    assert np.linalg.norm(Phi - ref) / np.linalg.norm(ref) < 1e-13


def test_general_form_equals_real_form_without_drift():
    rng = np.random.default_rng(4)
    s = rng.standard_normal((14, 9))
    s -= s.mean()
    a = DR.fixed_point("D2Q81", 5, 1.3, s, (0.0, 0.0))
    b = SP.fixed_point("D2Q81", 5, 1.3, s)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-13
