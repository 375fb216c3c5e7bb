"""GPU parity of the advection-diffusion variant (drifted equilibrium) and of
time-dependent runs from an equilibrium state, against the oracle."""
import sys

import numpy as np
import pytest

import paper_1504_05869_amd as lkp
from paper_1504_05869_amd import workloads as W
from oracle import drift as DR
from oracle import lattice as OL
from oracle import sweep as SW

pytestmark = pytest.mark.gpu

CASES = {"D1Q13": (7, (300,), (0.07,)), "D2Q81": (5, (31, 45), (0.05, -0.03)),
         "D2Q37": (5, (29, 35), (-0.04, 0.06)), "D2Q169": (7, (27, 33), (0.03, 0.02)),
         "D3Q111": (5, (9, 11, 13), (0.04, -0.02, 0.03))}


def say(*a):
    print("[gpu-drift]", *a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _source(shape, seed=11):
    return W.zero_mean(np.random.default_rng(seed).standard_normal(shape))


def _perm(lattice, order):
    """Oracle plane index of each of the library's velocities."""
    info = lkp.lattice_info(lattice, order)
    idx = {tuple(int(c) for c in v): i for i, v in enumerate(OL.get(lattice).v3())}
    return [idx[tuple(int(c) for c in v)] for v in info["v"]]


def _oracle_run(lattice, order, tau, s, u, sweeps, f0=None):
    p = SW.Problem(lattice, order, tau, s, drift=u)
    f = p.zero_state() if f0 is None else np.array(f0, dtype=np.float64)
    b, Phi = np.empty_like(f), np.empty(s.shape)
    for _ in range(sweeps):
        SW.sweep_c(p, f, b, Phi)
        f, b = b, f
    return Phi, f


@pytest.mark.parametrize("lattice", list(CASES))
@pytest.mark.parametrize("precision,bar", [("f64", 1e-13), ("f32", 2e-6)])
def test_drifted_sweeps_match_oracle(lattice, precision, bar):
    order, shape, u = CASES[lattice]
    s, tau, K = _source(shape), 1.4, 6
    say(lattice, precision, shape, "u", u)
    with lkp.Problem(s, lattice, order, tau_lb=tau, precision=precision, drift=u) as p:
        p.step(K)
        phi, f = p.phi_host(), p.populations()
    ref_phi, ref_f = _oracle_run(lattice, order, tau, s, u, K)
    assert rel_l2(phi, ref_phi) <= bar and rel_l2(f, ref_f[_perm(lattice, order)]) <= bar


@pytest.mark.parametrize("lattice", list(CASES))
def test_coefficients_match_oracle(lattice):
    order, shape, u = CASES[lattice]
    with lkp.Problem(_source(shape), lattice, order, tau_lb=1.4, drift=u) as p:
        phi, chi = p.coefficients()
    perm = _perm(lattice, order)
    rphi, rchi = DR.coefficients(OL.get(lattice), order, u)
    assert np.abs(phi - rphi[perm]).max() <= 4e-16 * np.abs(rphi).max()
    assert np.abs(chi - rchi[perm]).max() <= 4e-16 * np.abs(rchi).max()


@pytest.mark.parametrize("lattice,shape,tau,precision,bar", [
    ("D2Q81", (40, 48), 2.0, "f64", 1e-10), ("D2Q37", (36, 44), 1.5, "f64", 1e-10),
    ("D3Q111", (10, 12, 16), 1.2, "f64", 1e-10), ("D2Q81", (48, 40), 3.0, "f32_ir", 1e-9),
    ("D3Q111", (12, 10, 8), 1.5, "f32_ir", 1e-9)])
def test_converged_drifted_matches_spectral(lattice, shape, tau, precision, bar):
    """The steady state of the drifted scheme equals the exact complex
    spectral fixed point of lap Phi - (u/D).grad Phi = -s's lattice form."""
    order, _, u = CASES[lattice]
    s = W.zero_mean(W.gaussian_blobs(shape, 6, 1.5, 3))
    with lkp.Problem(s, lattice, order, tau_lb=tau, precision=precision, drift=u) as p:
        rep = p.solve(tol_rel_l2=bar / 10, check_every=50, max_sweeps=400000)
        phi = p.phi_host()
    ref = DR.fixed_point(lattice, order, tau, s, u)
    err = rel_l2(phi, ref)
    say(lattice, precision, "sweeps", rep["sweeps"], "true err", err)
    assert err <= bar


def test_drift_at_tau_one_sweeps_populations():
    order, shape, u = CASES["D2Q81"]
    s = _source(shape)
    with lkp.Problem(s, "D2Q81", order, tau_lb=1.0, drift=u) as p:
        assert p.info()["scalar_stencil"] == 0
        p.step(5)
        phi = p.phi_host()
    ref, _ = _oracle_run("D2Q81", order, 1.0, s, u, 5)
    assert rel_l2(phi, ref) <= 1e-13


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_drifted_in_place_equals_pull_bitwise(precision):
    order, shape, u = CASES["D3Q111"]
    s = _source(shape)
    out = []
    for ip in (False, True):
        with lkp.Problem(s, "D3Q111", order, tau_lb=1.3, precision=precision, drift=u,
                         in_place=ip) as p:
            p.step(7)
            out.append((p.phi_host(), p.populations()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("lattice,u", [("D2Q81", (0.05, 0.03)), ("D2Q81", (0.0, 0.0)),
                                       ("D3Q111", (0.04, -0.02, 0.03))])
def test_time_dependent_run_from_equilibrium(lattice, u):
    """Time-dependent use: from f*_i = phi_i Phi_0 (no source) the state after
    t sweeps equals the oracle's, value by value."""
    order = CASES[lattice][0]
    shape = (24, 32) if len(u) == 2 else (8, 10, 12)
    rng = np.random.default_rng(5)
    phi0 = rng.standard_normal(shape)
    s = np.zeros(shape)
    with lkp.Problem(s, lattice, order, tau_lb=1.3, drift=u, population_sweep=True) as p:
        p.set_equilibrium(phi0)
        p.step(40)
        phi = p.phi_host()
    sp = SW.Problem(lattice, order, 1.3, s, drift=u)
    f0 = sp.phi.reshape((-1,) + (1,) * len(shape)) * phi0[None]
    ref, _ = _oracle_run(lattice, order, 1.3, s, u, 40, f0=f0)
    assert rel_l2(phi, ref) <= 1e-13


def test_group_rejects_drifted_handle():
    order, shape, u = CASES["D2Q81"]
    g = lkp.Group("D2Q81", order, "f64")
    try:
        with lkp.Problem(_source(shape), "D2Q81", order, tau_lb=1.4, drift=u) as p:
            with pytest.raises(RuntimeError, match="drift"):
                g.add(p, tol_rel_l2=1e-8)
    finally:
        g.close()


def test_drifted_bf16_deviation_sweeps_match_oracle():
    """BF16 deviation storage with a drifted equilibrium: the plain deviation
    sweeps agree with the oracle's BF16 storage of the same scheme (bound as
    in tests/test_gpu_bf16dev.py: a quarter of the rounding effect)."""
    from oracle import bf16dev as B
    lattice, order, tau, shape, u = "D2Q81", 5, 2.5, (50, 70), (0.05, -0.03)
    s = W.zero_mean(np.random.default_rng(11).standard_normal(shape))
    K = 9
    with lkp.Problem(s, lattice, order, tau_lb=tau, precision="bf16dev_ir", drift=u) as p:
        p.step(K)
        a = p.phi_host()
    prob = SW.Problem(lattice, order, tau, s, drift=u)
    orc, _ = B.run(prob, K)
    exact, _ = SW.run(prob, K)
    effect = rel_l2(orc, exact)
    say("bf16dev drift: vs BF16 oracle", rel_l2(a, orc), "BF16 effect", effect)
    assert effect > 1e-7
    assert rel_l2(a, orc) <= 0.25 * effect
    assert rel_l2(a, exact) <= 1.25 * effect


def test_drifted_bf16_refinement_reaches_fixed_point():
    lattice, order, shape, u = "D2Q81", 5, (48, 40), (0.05, -0.03)
    s = W.zero_mean(W.gaussian_blobs(shape, 5, 1.5, 3))
    tau = 2.0
    with lkp.Problem(s, lattice, order, tau_lb=tau, precision="bf16dev_ir", drift=u) as p:
        rep = p.solve(tol_rel_l2=1e-9, check_every=20, max_sweeps=400000)
        phi = p.phi_host()
    err = rel_l2(phi, DR.fixed_point(lattice, order, tau, s, u))
    say("bf16dev drift solve: sweeps", rep["sweeps"], "outer", rep["outer"], "true err", err)
    assert err <= 1e-8


def test_drifted_in_place_refinement_equals_pull_bitwise():
    """FP32 + refinement with a drift, in place and with two buffers: the same
    answer bit for bit (the in-place layouts change only where values live)."""
    import os
    order, shape, u = 5, (40, 36), (0.05, -0.03)
    s = W.zero_mean(W.gaussian_blobs(shape, 5, 1.5, 9))
    old = os.environ.get("LKP_AUTOTUNE")
    os.environ["LKP_AUTOTUNE"] = "0"
    try:
        out = []
        for ip in (False, True):
            with lkp.Problem(s, "D2Q81", order, tau_lb=2.0, precision="f32_ir", drift=u,
                             in_place=ip) as p:
                rep = p.solve(tol_rel_l2=1e-10, check_every=50, max_sweeps=400000)
                out.append((p.phi_host(), rep["sweeps"]))
    finally:
        if old is None:
            os.environ.pop("LKP_AUTOTUNE")
        else:
            os.environ["LKP_AUTOTUNE"] = old
    assert out[0][1] == out[1][1] and np.array_equal(out[0][0], out[1][0])


def test_set_equilibrium_in_place_matches_two_buffers():
    order, u = 5, (0.05, 0.03)
    shape = (24, 32)
    phi0 = np.random.default_rng(6).standard_normal(shape)
    out = []
    for ip in (False, True):
        with lkp.Problem(np.zeros(shape), "D2Q81", order, tau_lb=1.3, drift=u,
                         population_sweep=True, in_place=ip) as p:
            p.set_equilibrium(phi0)
            p.step(12)
            out.append(p.phi_host())
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("precision", ["f64", "f32", "f32_ir"])
@pytest.mark.parametrize("in_place", [False, True])
def test_set_equilibrium_equals_host_built_populations(precision, in_place):
    """lkp_set_equilibrium (f*_i = phi_i Phi_0 formed on the device) stores
    exactly what lkp_set_populations stores for the same values built on the
    host from the handle's coefficients."""
    shape, u = (24, 32), (0.05, 0.03)
    phi0 = np.random.default_rng(8).standard_normal(shape)
    out = []
    for dev in (True, False):
        with lkp.Problem(np.zeros(shape), "D2Q81", 5, tau_lb=1.3, drift=u, precision=precision,
                         population_sweep=True, in_place=in_place) as p:
            if dev:
                p.set_equilibrium(phi0)
            else:
                c, _ = p.coefficients()
                p.set_populations(c[:, None, None] * phi0[None])
            f0 = p.populations()
            if precision == "f32_ir":  # refinement handles are driven by lkp_solve only
                out.append((f0, None))
                continue
            p.step(6)
            out.append((f0, p.phi_host()))
    assert np.array_equal(out[0][0], out[1][0])
    if out[0][1] is not None:
        assert np.array_equal(out[0][1], out[1][1])


def test_set_equilibrium_refused_by_stencil_form():
    with lkp.Problem(np.zeros((16, 16)), "D2Q81", 5, tau_lb=1.0) as p:
        with pytest.raises(lkp.LkpError) as ei:
            p.set_equilibrium(np.ones((16, 16)))
        assert ei.value.name == "LKP_ERR_UNSUPPORTED"
