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


def test_fp32_evaluation_stays_close_to_fp64_evaluation():
    """The FP32-arithmetic emulation (rounding decisions taken on FP32 values)
    differs from the FP64 one only by rounding-decision flips: far less than
    the BF16 effect itself; velocity grouping of the FP64 moment sum hardly
    matters."""
    s = W.zero_mean(np.random.default_rng(11).standard_normal((30, 40)))
    p = SW.Problem("D2Q81", 5, 2.5, s)
    S32 = p.S.astype(np.float32)
    a, _ = B.run(p, 9, S=S32, fp32_groups=1)
    b, _ = B.run(p, 9, S=S32.astype(np.float64))
    e, _ = SW.run(p, 9)
    effect = np.linalg.norm(b - e) / np.linalg.norm(e)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 0.1 * effect
    c, _ = B.run(p, 9, S=S32, fp32_groups=4)
    assert np.linalg.norm(a - c) / np.linalg.norm(a) <= 1e-3 * effect
