"""GPU tests of in-place single-buffer sweeps (LKP_FLAG_IN_PLACE): every result
equals the two-buffer pull sweep's, bit for bit."""
import os
import sys

import numpy as np
import pytest

import paper_1504_05869_amd as lkp
from paper_1504_05869_amd import workloads as W
from oracle import sweep as SW

pytestmark = pytest.mark.gpu

SETS = {"D1Q13": (7, (300,)), "D2Q5": (1, (45, 70)), "D2Q9": (3, (33, 40)),
        "D2Q25": (3, (37, 66)), "D2Q81": (5, (50, 70)), "D2Q169": (7, (41, 77)),
        "D3Q111": (5, (13, 19, 37)), "D2Q37": (5, (43, 50)), "D2Q77": (7, (39, 66)),
        "D3Q107": (5, (11, 17, 29))}


def say(*a):
    print("[gpu-inplace]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def same_split():
    """Both handles use the default velocity-group split (in place is never
    tuned), so the moment sums run in the same order."""
    old = os.environ.get("LKP_AUTOTUNE")
    os.environ["LKP_AUTOTUNE"] = "0"
    yield
    if old is None:
        os.environ.pop("LKP_AUTOTUNE", None)
    else:
        os.environ["LKP_AUTOTUNE"] = old


def _src(shape, seed=1):
    return W.zero_mean(np.random.default_rng(seed).standard_normal(shape))


def _run(s, lattice, order, tau, precision, in_place, sweeps):
    with lkp.Problem(s, lattice, order, tau_lb=tau, precision=precision, in_place=in_place) as p:
        assert p.info()["in_place"] == int(in_place)
        p.step(sweeps)
        return p.phi_host(), p.populations(), p.residual()


@pytest.mark.parametrize("lattice", list(SETS))
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("sweeps", [7, 8])
def test_in_place_equals_pull_bitwise(lattice, precision, sweeps):
    order, shape = SETS[lattice]
    s = _src(shape)
    a = _run(s, lattice, order, 1.7, precision, True, sweeps)
    b = _run(s, lattice, order, 1.7, precision, False, sweeps)
    assert np.array_equal(a[0], b[0])          # Phi
    assert np.array_equal(a[1], b[1])          # populations, remapped to the pull layout
    for k in ("max_change", "l2_change", "phi_l2", "mass"):
        assert a[2][k] == b[2][k], k
    if precision == "f64":
        assert a[2]["pop_residual_l2"] == b[2]["pop_residual_l2"]
    ref, _ = SW.run(SW.Problem(lattice, order, 1.7, s), sweeps)
    err = float(np.linalg.norm(a[0] - ref) / np.linalg.norm(ref))
    say(lattice, precision, sweeps, "vs oracle", err)
    assert err <= (1e-13 if precision == "f64" else 2e-6)


@pytest.mark.parametrize("lattice,shape", [("D2Q81", (3, 130)), ("D3Q111", (2, 3, 5)),
                                           ("D2Q169", (4, 5))])
def test_in_place_small_grids(lattice, shape):
    order = SETS[lattice][0]
    s = _src(shape, 3)
    a = _run(s, lattice, order, 2.2, "f64", True, 5)
    b = _run(s, lattice, order, 2.2, "f64", False, 5)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("precision", ["f64", "f32_ir"])
def test_in_place_solve_bitwise(precision):
    s = W.zero_mean(W.gaussian_blobs((64, 48), 5, 1.5, 2))
    out = []
    for ip in (True, False):
        with lkp.Problem(s, "D2Q81", 5, knudsen=0.1, precision=precision, in_place=ip) as p:
            rep = p.solve(tol_rel_l2=1e-10, check_every=20, max_sweeps=200000)
            out.append((rep["sweeps"], rep["outer"], p.phi_host()))
    say(precision, "sweeps", out[0][0], out[1][0], "outer", out[0][1], out[1][1])
    assert out[0][0] == out[1][0] and out[0][1] == out[1][1]
    assert np.array_equal(out[0][2], out[1][2])


def test_in_place_set_populations_roundtrip():
    s = _src((20, 30), 5)
    f0 = np.random.default_rng(6).standard_normal((81, 20, 30)) * 1e-3
    res = []
    for ip in (True, False):
        with lkp.Problem(s, "D2Q81", 5, tau_lb=2.5, in_place=ip) as p:
            p.set_populations(f0)
            assert np.array_equal(p.populations(), f0)
            p.step(3)
            res.append((p.phi_host(), p.populations()))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])


def test_in_place_rejections():
    s = _src((16, 16), 4)
    g = lkp.Group("D2Q25", 3, "f64")
    with lkp.Problem(s, "D2Q25", 3, tau_lb=2.0, in_place=True) as p:
        with pytest.raises(lkp.LkpError) as ei:
            g.add(p, tol_rel_l2=1e-8)
        assert ei.value.name == "LKP_ERR_UNSUPPORTED"
    g.close()
    with pytest.raises(lkp.LkpError) as ei:
        lkp.Problem(s, "D2Q25", 3, tau_lb=2.0, precision="bf16dev_ir", in_place=True)
    assert ei.value.name == "LKP_ERR_UNSUPPORTED"
