"""BF16 deviation storage of the post-collision state (test infrastructure only).

An ablation of the storage precision, not of the scheme: the sweep is the
discrete BGK iteration of ``oracle.sweep`` (stream, moment, collide + source,
Sec. 4 and 5), but between sweeps the post-collision populations are kept as

    f*_i(x) = phi_i Phi(x) + n_i(x)

with Phi, the moment of the populations streamed into x, rounded to FP32 and
the deviation n_i rounded to BF16 (8 significant bits, round to nearest, ties
to even).  One sweep therefore reads

    f_i(x)  = phi_i Phi(x - v_i) + n_i(x - v_i)
    Phi'(x) = sum_i f_i(x),                 stored as fp32(Phi')
    n'_i(x) = bf16((1 - omega) (f_i(x) - phi_i fp32(Phi'(x))) + chi_i S(x))

where the argument of bf16() is exactly f*'_i - phi_i fp32(Phi') for the
collision of the scheme.  All arithmetic is FP64; only the stored values are
rounded.  With the rounding switched off the iteration is the scheme's sweep
in other variables (pinned in tests against ``oracle.sweep``).
"""
from __future__ import annotations

import numpy as np

from . import sweep as SW

# BF16: 8 significant bits (7 stored), the exponent range of FP32.
_BF16_BITS = 8
_MIN_NORMAL_EXP = -125     # frexp exponent of 2^-126, the smallest normal value
_SUBNORMAL_STEP = 2.0 ** (-126 - (_BF16_BITS - 1))


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Nearest BF16 value (ties to even), from the format's definition:
    keep 8 significant bits of a normal number, a fixed step of 2^-133 below
    2^-126.  Values are returned as float64."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                       # x = m 2^e, 1/2 <= |m| < 1
    scale = float(2 ** _BF16_BITS)
    normal = np.ldexp(np.rint(m * scale) / scale, e)   # np.rint: half to even
    sub = np.rint(x / _SUBNORMAL_STEP) * _SUBNORMAL_STEP
    return np.where(e >= _MIN_NORMAL_EXP, normal, sub)


def round_fp32(x: np.ndarray) -> np.ndarray:
    """Nearest FP32 value (the library cast rounds to nearest even)."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def _identity(x):
    return np.asarray(x, dtype=np.float64)


def sweep(p: SW.Problem, n: np.ndarray, Phi: np.ndarray, S: np.ndarray | None = None,
          rounding: bool = True):
    """One sweep on the stored state (n, Phi); returns the new (n, Phi).

    S is the scaled source (default: the problem's).  rounding=False keeps
    every stored value in FP64."""
    rb, rf = (round_bf16, round_fp32) if rounding else (_identity, _identity)
    S = p.S if S is None else S
    axes = tuple(range(-1, -p.lat.dim - 1, -1))          # x, y, z -> last axes
    f = np.empty((p.lat.Q,) + p.shape)
    for i, v in enumerate(p.lat.v):
        shift = tuple(int(c) for c in v)
        f[i] = p.phi[i] * np.roll(Phi, shift=shift, axis=axes) + np.roll(n[i], shift=shift, axis=axes)
    Phi_new = np.zeros(p.shape)
    for i in range(p.lat.Q):
        Phi_new = Phi_new + f[i]
    Phi_s = rf(Phi_new)
    n_new = np.empty_like(f)
    for i in range(p.lat.Q):
        n_new[i] = rb((1.0 - p.omega) * (f[i] - p.phi[i] * Phi_s) + p.chi[i] * S)
    return n_new, Phi_s


def run(p: SW.Problem, sweeps: int, S: np.ndarray | None = None, rounding: bool = True):
    """`sweeps` sweeps from rest (n = 0, Phi = 0); returns (Phi, n)."""
    n = np.zeros((p.lat.Q,) + p.shape)
    Phi = np.zeros(p.shape)
    for _ in range(sweeps):
        n, Phi = sweep(p, n, Phi, S, rounding)
    return Phi, n
