"""GPU tests of the BF16 deviation-storage ablation (precision "bf16dev_ir")."""
import sys

import numpy as np
import pytest

import paper_1504_05869_amd as lkp
from paper_1504_05869_amd import workloads as W
from oracle import bf16dev as B
from oracle import lattice as OL
from oracle import spectral as SP
from oracle import sweep as SW

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-bf16dev]", *a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def check_against_bf16_oracle(a, prob, K, tag):
    """GPU Phi after K plain deviation sweeps from rest against the oracle's
    BF16 storage (FP64 arithmetic, only the stored values rounded).

    Both sides round the same values to BF16 (unit roundoff u = 2^-8), so
    they differ only where the GPU's FP32 arithmetic noise (2^-24 relative to
    the populations) moves a value across a BF16 rounding boundary.  A flipped
    decision costs one BF16 step (2u |n|) where an agreeing one costs a
    rounding error of about u |n| / sqrt(3) rms, so with a fraction q of flips
    the rms disagreement is about 2 sqrt(3 q) times the rounding effect
    itself (oracle vs unrounded scheme).  The bound, a quarter of that effect,
    allows q up to 0.5 %; a missing term or a wrong rounding would leave the
    GPU many times the effect away."""
    orc, _ = B.run(prob, K)
    exact, _ = SW.run(prob, K)
    effect = rel_l2(orc, exact)
    d = rel_l2(a, orc)
    say(tag, "vs BF16 oracle", d, "BF16 effect (oracle vs unrounded scheme)", effect,
        "ratio", d / effect, "GPU vs unrounded", rel_l2(a, exact))
    assert effect > 1e-7                     # the rounding is visible at all
    assert d <= 0.25 * effect
    assert rel_l2(a, exact) <= 1.25 * effect


@pytest.mark.parametrize("lattice,order,tau,shape", [
    ("D2Q25", 3, 3.0, (37, 66)), ("D2Q81", 5, 2.5, (50, 70)), ("D2Q169", 7, 4.0, (41, 77)),
    ("D3Q111", 5, 1.7, (13, 19, 37)), ("D1Q13", 7, 3.0, (300,)), ("D2Q81", 5, 6.0, (3, 130)),
    ("D3Q107", 5, 2.2, (12, 15, 21))])
def test_plain_deviation_sweeps_match_oracle(lattice, order, tau, shape):
    """K plain sweeps with BF16 deviation storage from rest (lkp_step on a
    bf16dev_ir handle) against the oracle's BF16 storage of the same scheme."""
    s = W.zero_mean(np.random.default_rng(11).standard_normal(shape))
    K = 9
    with lkp.Problem(s, lattice, order, tau_lb=tau, precision="bf16dev_ir") as p:
        p.step(K)
        a = p.phi_host()
    check_against_bf16_oracle(a, SW.Problem(lattice, order, tau, s), K, f"{lattice} {shape}")


@pytest.mark.parametrize("lattice,order,shape,kn", [("D2Q81", 5, (48, 40), 0.1),
                                                    ("D3Q111", 5, (12, 10, 16), 0.2)])
def test_bf16dev_refinement_reaches_fixed_point(lattice, order, shape, kn):
    s = W.zero_mean(W.gaussian_blobs(shape, 5, 1.5, 3))
    tau = OL.tau_from_knudsen(kn, OL.get(lattice), min(shape))
    ref = SP.fixed_point(lattice, order, tau, s)
    with lkp.Problem(s, lattice, order, knudsen=kn, precision="bf16dev_ir") as p:
        rep = p.solve(tol_rel_l2=1e-9, check_every=20, max_sweeps=400000)
        phi = p.phi_host()
    err = rel_l2(phi, ref)
    say(lattice, shape, "sweeps", rep["sweeps"], "outer", rep["outer"], "true err", err)
    assert err <= 1e-8


def test_bf16dev_rejections():
    s = W.zero_mean(np.random.default_rng(4).standard_normal((16, 16)))
    with pytest.raises(lkp.LkpError) as ei:
        lkp.Problem(s, "D2Q25", 3, tau_lb=1.0, precision="bf16dev_ir")
    assert ei.value.name == "LKP_ERR_UNSUPPORTED"
    with pytest.raises(lkp.LkpError) as ei:
        lkp.Group("D2Q25", 3, "bf16dev_ir")
    assert ei.value.name == "LKP_ERR_UNSUPPORTED"
    # at tau_lb = 1 the population form still takes it
    with lkp.Problem(s, "D2Q25", 3, tau_lb=1.0, precision="bf16dev_ir", population_sweep=True) as p:
        p.step(3)
        assert np.isfinite(p.phi_host()).all()
