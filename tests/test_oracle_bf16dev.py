"""Pins of the BF16 deviation-storage oracle (CPU)."""
import numpy as np
import pytest
import torch

from oracle import bf16dev as B
from oracle import sweep as SW
from paper_1504_05869_amd import workloads as W


def test_round_bf16_matches_torch_cast():
    """Independent implementation: torch's float32 -> bfloat16 conversion
    (round to nearest even), on FP32 values over the whole exponent range,
    subnormals included."""
    rng = np.random.default_rng(0)
    x = rng.standard_normal(200000) * np.exp2(rng.uniform(-140, 120, 200000))
    x = x.astype(np.float32).astype(np.float64)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(B.round_bf16(x), ref)


def test_round_bf16_ties_to_even():
    u = 2.0 ** -7                                    # BF16 spacing in [1, 2)
    assert B.round_bf16(np.array([1 + u / 2]))[0] == 1.0          # tie, 1.0 is even
    assert B.round_bf16(np.array([1 + 3 * u / 2]))[0] == 1 + 2 * u  # tie, 1 + 2u is even
    assert B.round_bf16(np.array([1 + u / 2 + 2.0 ** -30]))[0] == 1 + u
    assert B.round_bf16(np.array([-(1 + u / 2)]))[0] == -1.0
    assert B.round_bf16(np.array([0.0]))[0] == 0.0


def test_round_bf16_error_bound_and_idempotence():
    x = np.random.default_rng(1).standard_normal(10000) * 1e3
    r = B.round_bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x))   # unit roundoff of 8 bits
    assert np.array_equal(B.round_bf16(r), r)


@pytest.mark.parametrize("lattice,order,tau,shape", [("D2Q81", 5, 2.5, (12, 17)),
                                                     ("D3Q111", 5, 1.7, (6, 7, 9)),
                                                     ("D1Q13", 7, 3.0, (40,))])
def test_deviation_form_without_rounding_is_the_scheme(lattice, order, tau, shape):
    """Stored as phi_i Phi + n_i but not rounded, the iteration is the scheme's
    sweep in other variables: Phi agrees with the C oracle after K sweeps."""
    s = W.zero_mean(np.random.default_rng(2).standard_normal(shape))
    p = SW.Problem(lattice, order, tau, s)
    ref, _ = SW.run(p, 7)
    phi, _ = B.run(p, 7, rounding=False)
    assert np.max(np.abs(phi - ref)) <= 1e-13 * np.max(np.abs(ref))
    # planted mistake: a source term off by a factor breaks the agreement
    bad, _ = B.run(p, 7, S=2.0 * p.S, rounding=False)
    assert np.max(np.abs(bad - ref)) > 1e-3 * np.max(np.abs(ref))


def test_rounding_is_active_and_small():
    s = W.zero_mean(np.random.default_rng(3).standard_normal((20, 24)))
    p = SW.Problem("D2Q81", 5, 4.0, s)
    exact, _ = B.run(p, 10, rounding=False)
    rounded, n = B.run(p, 10)
    err = np.linalg.norm(rounded - exact) / np.linalg.norm(exact)
    assert 1e-7 < err < 1e-2
    assert np.array_equal(B.round_bf16(n), n)     # the stored deviations are BF16 values


def test_rounding_stays_inside_its_envelope():
    """One sweep from a common stored state: the new Phi carries one FP32
    rounding, |dPhi| <= 2^-24 |Phi|, and each new deviation one BF16 rounding
    of an argument that differs from the unrounded one only through that Phi,
    so |dn_i| <= 2^-8 |n_i| + (1 + 2^-8) |1 - omega| |phi_i| |dPhi|.  Checked
    value by value, and the unrounded sweep is the scheme's sweep of the
    populations phi_i Phi + n_i."""
    rng = np.random.default_rng(12)
    s = W.zero_mean(rng.standard_normal((14, 18)))
    p = SW.Problem("D2Q81", 5, 2.5, s)
    Phi0 = B.round_fp32(rng.standard_normal(p.shape))
    n0 = B.round_bf16(0.1 * rng.standard_normal((p.lat.Q,) + p.shape))
    n_r, Phi_r = B.sweep(p, n0, Phi0)
    n_e, Phi_e = B.sweep(p, n0, Phi0, rounding=False)
    u8, u24 = 2.0 ** -8, 2.0 ** -24
    dPhi = np.abs(Phi_r - Phi_e)
    assert np.all(dPhi <= u24 * np.abs(Phi_e))
    bound = u8 * np.abs(n_e) + (1 + u8) * abs(1 - p.omega) * np.abs(p.phi)[:, None, None] * dPhi[None]
    assert np.all(np.abs(n_r - n_e) <= bound * (1 + 1e-12))
    assert np.any(n_r != n_e)                       # the rounding is active
    # the inputs were already representable: the unrounded sweep's Phi is the
    # scheme's Phi of the populations phi_i Phi0 + n0
    f0 = p.phi[:, None, None] * Phi0[None] + n0
    out = np.empty_like(f0)
    Phi_c = np.empty(p.shape)
    SW.sweep_c(p, np.ascontiguousarray(f0), out, Phi_c)
    assert np.max(np.abs(Phi_c - Phi_e)) <= 1e-13 * np.max(np.abs(Phi_e))
