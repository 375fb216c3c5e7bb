"""Velocity-set generator from the quadrature conditions (test infrastructure only).

Sec. 4 reads the scheme's requirements as orthogonality conditions on the
discrete velocities (Eq. quadrature in 1D, Eq. quad3 in 3D): weighted sums over
the set must reproduce the Gaussian moments of w(v) up to the degree the
expansion order needs, and it notes that the same procedure is a systematic way
to obtain weights and velocities for a wanted accuracy.  This module does that
search for sets symmetric under axis permutations and sign flips:

* a set is a union of integer *shells* (orbits of such a vector), each with one
  weight;
* by symmetry every odd moment vanishes, and the even moments up to degree D
  reduce to one equation per *class* x1^a1 ... xd^ad with a1 >= ... >= ad even;
* with one shell fewer than classes, the equations fix c_s^2 as a root of the
  determinant of the augmented system (the conditions must be consistent), and
  then the weights;
* a set is admissible when every weight is positive.

``search`` enumerates shell subsets (the origin always included) in order of
increasing velocity count and returns the admissible ones of the smallest
count.  The scan over c_s^2 uses float64 determinants; roots are refined and
the weights solved with mpmath at 50 digits.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import mpmath as mp
import numpy as np
from threadpoolctl import threadpool_limits

DPS = 50


def _dfact(n: int) -> int:
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def classes(dim: int, degree: int):
    """Even exponent classes (a1 >= ... >= ad >= 0, all even), total <= degree."""
    out = []

    def rec(prefix, left, cap):
        if len(prefix) == dim:
            out.append(tuple(prefix))
            return
        for a in range(min(left, cap), -1, -2):
            if a % 2 == 0:
                rec(prefix + [a], left - a, a)

    rec([], degree - degree % 2, degree)
    return sorted(out, key=lambda e: (sum(e), [-x for x in e]))


def shells(dim: int, maxc: int):
    """Shell representatives (sorted descending absolute components) up to maxc."""
    reps = set()
    for v in itertools.product(range(maxc + 1), repeat=dim):
        reps.add(tuple(sorted(v, reverse=True)))
    return sorted(reps, key=lambda s: (sum(x * x for x in s), s))


def orbit(rep):
    """All signed permutations of a shell representative (distinct vectors)."""
    out = set()
    for p in itertools.permutations(rep):
        for signs in itertools.product((1, -1), repeat=len(rep)):
            out.add(tuple(s * x for s, x in zip(signs, p)))
    return sorted(out)


def _shell_moments(reps, cls):
    """M[r][j] = sum over the orbit of shell j of the class-r monomial (exact ints)."""
    M = np.zeros((len(cls), len(reps)), dtype=object)
    for j, rep in enumerate(reps):
        for v in orbit(rep):
            for r, e in enumerate(cls):
                m = 1
                for x, a in zip(v, e):
                    m *= x ** a
                M[r, j] += m
    return M


def gauss_moment(e, t):
    """Moment of the normalised Gaussian of variance t: prod (a-1)!! t^(a/2)."""
    m = 1
    for a in e:
        m *= _dfact(a - 1)
    return m * t ** (sum(e) // 2)


@dataclass
class Found:
    dim: int
    degree: int
    reps: list          # shell representatives
    cs2: object         # mpmath mpf
    shell_weights: list # mpmath mpf per shell
    q: int              # number of velocities

    def velocities(self):
        v, w = [], []
        for rep, W in zip(self.reps, self.shell_weights):
            for x in orbit(rep):
                v.append(x)
                w.append(W)
        return np.array(v, dtype=np.int64), w


T_GRID = np.linspace(0.05, 3.0, 600)


def _rhs_grid(cls, t_grid):
    return np.array([[float(gauss_moment(e, t)) for e in cls] for t in t_grid])


def solve_subset(reps, cls, t_grid=None, M=None, rhs=None):
    """Admissible (c_s^2, weights) pairs of one shell subset (|reps| = |cls| - 1)."""
    if M is None:
        M = _shell_moments(reps, cls)
    Mf = M.astype(np.float64)
    if np.linalg.matrix_rank(Mf / np.abs(Mf).max(axis=1, keepdims=True)) < Mf.shape[1]:
        return []  # dependent shell columns: the weights are not determined
    if t_grid is None:
        t_grid = T_GRID
    if rhs is None:
        rhs = _rhs_grid(cls, t_grid)
    stack = np.empty((len(t_grid),) + (Mf.shape[0], Mf.shape[1] + 1))
    stack[:, :, :-1] = Mf
    stack[:, :, -1] = rhs
    vals = np.linalg.det(stack)
    found = []
    for k in range(len(t_grid) - 1):
        if not (np.isfinite(vals[k]) and np.isfinite(vals[k + 1])) or vals[k] * vals[k + 1] > 0:
            continue
        with mp.workdps(DPS):
            Mm = mp.matrix([[mp.mpf(int(M[r, j])) for j in range(M.shape[1])] for r in range(M.shape[0])])

            def det_aug(t):
                A = mp.matrix(Mm.rows, Mm.cols + 1)
                for i in range(Mm.rows):
                    for j in range(Mm.cols):
                        A[i, j] = Mm[i, j]
                    A[i, Mm.cols] = gauss_moment(cls[i], t)
                return mp.det(A)
            try:
                t = mp.findroot(det_aug, (mp.mpf(t_grid[k]), mp.mpf(t_grid[k + 1])), solver="anderson")
            except (ValueError, ZeroDivisionError, TypeError):
                continue
            rhs = mp.matrix([gauss_moment(e, t) for e in cls])
            try:  # dependent shell columns: no unique weights, not admissible
                W = mp.lu_solve(Mm.T * Mm, Mm.T * rhs)
            except ZeroDivisionError:
                continue
            resid = mp.norm(Mm * W - rhs)
            if resid < mp.mpf(10) ** (-30) and all(W[j] > 0 for j in range(len(reps))):
                found.append((t, [W[j] for j in range(len(reps))]))
    return found


def max_amplification(v: np.ndarray, phi: np.ndarray, tau_lb: float, nk: int) -> float:
    """Largest modulus of the one-sweep amplification over an nk^d grid of
    wavevectors (Fourier analysis of the scheme's sweep, Sec. 4 and 5): for
    mode k the post-collision populations map by (1 - omega) E + omega phi 1^T E,
    E = diag(exp(-i k . v_j)).  v: (Q, d) integer velocities, phi: (Q,)."""
    V = np.asarray(v, dtype=np.float64)
    om = 1.0 / tau_lb
    worst = 0.0
    ks = np.linspace(0.0, 2.0 * np.pi, nk, endpoint=False)
    # many small eigenproblems: BLAS threads only contend here
    with threadpool_limits(1):
        for k in itertools.product(ks, repeat=V.shape[1]):
            e = np.exp(-1j * (V @ np.array(k)))
            M = (1.0 - om) * np.diag(e) + om * np.outer(phi, e)
            worst = max(worst, float(np.max(np.abs(np.linalg.eigvals(M)))))
    return worst


def spectral_radius(found: Found, order: int, tau_lb: float, nk: int = 8) -> float:
    """``max_amplification`` of the order-N scheme on a generated set, with
    the Hermite shape phi_i of the order."""
    from . import lattice as L
    v, w = found.velocities()
    with mp.workdps(30):
        t = found.cs2
        phi = []
        for vec, wi in zip(v, w):
            r2 = mp.mpf(int(sum(int(c) * int(c) for c in vec))) / t
            p, _ = L.shape_factors(r2, found.dim, order)
            phi.append(float(wi * p))
    return max_amplification(v, np.array(phi), tau_lb, nk)


def lattice_spectral_radius(lattice: str, order: int, tau_lb: float, nk: int = 8) -> float:
    """``max_amplification`` of the order-N scheme on a named set of
    ``oracle.lattice``."""
    from . import lattice as L
    lat = L.get(lattice)
    phi, _ = L.coefficients(lat, order)
    return max_amplification(lat.v3()[:, :lat.dim], phi, tau_lb, nk)


def stable(found: Found, order: int, taus=(1.0, 100.0), nk: int = 8, tol: float = 1e-9) -> bool:
    """No growing mode at the given relaxation times (the checkerboard mode and
    the rest of the nk^d grid)."""
    return all(spectral_radius(found, order, t, nk) <= 1.0 + tol for t in taus)


def search(dim: int, degree: int, maxc: int, limit: int | None = None, require_stable_order: int = 0):
    """Smallest admissible sets exact for every monomial of degree <= degree + 1.

    Returns the list of sets (Found) of the smallest velocity count among shell
    subsets with components <= maxc, or [] if none exists.  With
    require_stable_order = N, a set is admissible only if the order-N scheme
    on it has no growing mode (``stable``)."""
    cls = classes(dim, degree)
    cand = shells(dim, maxc)
    origin, others = cand[0], cand[1:]
    need = len(cls) - 2                       # shells besides the origin
    sizes = {r: len(orbit(r)) for r in cand}
    cols = {r: _shell_moments([r], cls)[:, 0] for r in cand}
    rhs = _rhs_grid(cls, T_GRID)
    subsets = sorted(itertools.combinations(others, need),
                     key=lambda c: (1 + sum(sizes[r] for r in c), [sum(x * x for x in r) for r in c]))
    best_q, out = None, []
    for k, sub in enumerate(subsets):
        if limit is not None and k >= limit:
            break
        q = 1 + sum(sizes[r] for r in sub)
        if best_q is not None and q > best_q:
            break
        reps = [origin] + list(sub)
        M = np.column_stack([cols[r] for r in reps])
        for t, W in solve_subset(reps, cls, M=M, rhs=rhs):
            f = Found(dim, degree, reps, t, W, q)
            if require_stable_order and not stable(f, require_stable_order):
                continue
            best_q = q
            out.append(f)
    return out
