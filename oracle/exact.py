"""Exact-arithmetic checks of the lattice constants (test infrastructure only).

The sound speed c_s^2 = t is kept as a symbol.  Because the moment-matching
system of Eq. (quadrature)/(quad3) has a constant rational matrix and a
right-hand side polynomial in t, every weight is a polynomial in t with
rational coefficients.  The condition that fixes c_s^2 (one moment beyond the
weights' own equations) is then a polynomial P(t); the admissible c_s^2 is a
root of one of its irreducible factors, and any identity that holds on the
lattice must reduce to zero modulo that factor.  This is exact algebraic
arithmetic: no rounding anywhere.

D1Q13 is the exception: the Appendix prints c_s itself, so t is the square of
that decimal, a rational number, and everything is plain Fraction arithmetic.

Checked identities (Sec. 4, after Eqs. omega:eq and chi:eq, and Eq. CON),
for every monomial v^a of total degree n <= N:
    sum_i phi_i v_i^a = 1 (n=0), 0 (n=1), c_s^2 delta_ab (n=2), 0 (2<n<=N)
    sum_i chi_i v_i^a = 1 (n=0), 0 (0<n<=N)
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import sympy as sp

from . import lattice as L

t = sp.Symbol("t")


def _dfact(n):
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def _gauss(exps):
    """Gaussian moment of prod x^e as a polynomial in t = c_s^2."""
    r = sp.Integer(1)
    for e in exps:
        if e % 2:
            return sp.Integer(0)
        r *= _dfact(e - 1) * t ** (e // 2)
    return r


def _shell_weights(shells, classes, moment_of_shell):
    """Solve len(shells) moment equations exactly; weights as polys in t."""
    n = len(shells)
    A = sp.Matrix(n, n, lambda r, j: moment_of_shell(shells[j], classes[r]))
    b = sp.Matrix(n, 1, lambda r, _: _gauss(classes[r]))
    W = A.LUsolve(b)
    return [sp.expand(x) for x in W]


def _select_factor(poly, approx):
    """Irreducible factor of poly (in t) that vanishes at the numeric root."""
    _, facs = sp.factor_list(sp.Poly(poly, t))
    best = None
    for f, _ in facs:
        val = abs(complex(f.as_expr().subs(t, approx)))
        if best is None or val < best[0]:
            best = (val, f)
    return best[1]


class ExactLattice:
    """Velocities, weights as polynomials in t, and the modulus for t."""

    def __init__(self, name):
        num = L.get(name)
        self.name = name
        self.dim = num.dim
        self.v = [tuple(int(c) for c in row) for row in num.v]
        self.modulus = None          # sympy Poly, or None when t is rational
        self.t_value = None          # rational t when modulus is None
        if name in ("D2Q5", "D2Q9"):
            self.t_value = sp.Rational(1, 3)
            self.w = []
            for vec in self.v:
                r2 = vec[0] ** 2 + vec[1] ** 2
                if name == "D2Q5":
                    self.w.append(sp.Rational(1, 3) if r2 == 0 else sp.Rational(1, 6))
                else:
                    self.w.append({0: sp.Rational(4, 9), 1: sp.Rational(1, 9),
                                   2: sp.Rational(1, 36)}[r2])
            return
        if name in L.SPEEDS_1D or name in ("D2Q25", "D2Q81", "D2Q169"):
            base = {"D2Q25": "D1Q5", "D2Q81": "D1Q9", "D2Q169": "D1Q13"}.get(name, name)
            speeds = L.SPEEDS_1D[base]
            shells = sorted({abs(s) for s in speeds})
            classes = [(2 * k,) for k in range(len(shells))]

            def mom(s, e):
                m = 1 if s == 0 else 2
                return m * sp.Integer(s) ** e[0]
            W = _shell_weights(shells, classes, mom)
            w1 = {s: W[j] for j, s in enumerate(shells)}
            if base == "D1Q5":
                self.modulus = sp.Poly(5 * t ** 2 - 10 * t + 3, t)
                extra = None
            elif base == "D1Q13":
                self.t_value = sp.Rational(str(Fraction(L.D1Q13_CS))) ** 2
                extra = None
            else:  # D1Q9: the degree-10 moment fixes t
                k = len(shells)
                extra = sp.expand(sum(w1[abs(s)] * sp.Integer(s) ** (2 * k)
                                      for s in speeds) - _gauss((2 * k,)))
                self.modulus = _select_factor(extra, float(L.get(base).c2_mp))
            if self.t_value is not None:
                w1 = {s: sp.expand(x.subs(t, self.t_value)) for s, x in w1.items()}
            if self.dim == 1:
                self.w = [w1[abs(vec[0])] for vec in self.v]
            else:
                self.w = [sp.expand(w1[abs(vec[0])] * w1[abs(vec[1])]) for vec in self.v]
            return
        if name == "D3Q111" or name in L.GENERATED_SHELLS:
            if name == "D3Q111":
                shells = [b for b, _ in L.D3Q111_SHELLS]
                classes = L._D3_CLASSES
            else:
                from . import generator as G
                shells = L.GENERATED_SHELLS[name]
                classes = G.classes(len(shells[0]), L.generated_degree(name))
            orbits = [L._orbit(b) for b in shells]
            ns = len(shells)

            def mom(j, e):
                r = sp.Integer(0)
                for vec in orbits[j]:
                    m = sp.Integer(1)
                    for x, a in zip(vec, e):
                        m *= sp.Integer(x) ** a
                    r += m
                return r
            idx = list(range(ns))
            # len(shells) independent classes fix the weights, the remaining
            # one fixes t
            for drop in reversed(range(len(classes))):
                use = [c for k, c in enumerate(classes) if k != drop]
                A = sp.Matrix(ns, ns, lambda r, j: mom(idx[j], use[r]))
                if A.rank() == ns:
                    break
            W = _shell_weights(idx, use, mom)
            e = classes[drop]
            extra = sp.expand(sum(W[j] * mom(j, e) for j in idx) - _gauss(e))
            self.modulus = _select_factor(extra, float(L.get(name).c2_mp))
            wshell = {shells[j]: W[j] for j in idx}
            self.w = []
            for vec in self.v:
                key = tuple(sorted((abs(c) for c in vec), reverse=True))
                self.w.append(wshell[key])
            return
        raise KeyError(name)

    def reduce(self, expr):
        """Exact zero test of a rational expression in t on this lattice."""
        expr = sp.together(sp.expand(expr))
        if self.modulus is None:
            return sp.simplify(expr.subs(t, self.t_value)) == 0
        num, _ = sp.fraction(expr)
        num = sp.Poly(sp.expand(num), t)
        return num.rem(self.modulus).is_zero

    def weight_values(self, dps=50):
        """Numeric weights at the admissible t (for comparison with lattice.py)."""
        import mpmath as mp
        with mp.workdps(dps):
            if self.modulus is None:
                tv = mp.mpf(sp.Rational(self.t_value).p) / sp.Rational(self.t_value).q
            else:
                roots = [r for r in mp.polyroots([int(c) if c.is_integer else mp.mpf(c.p) / c.q
                                                  for c in self.modulus.all_coeffs()],
                                                 maxsteps=200, extraprec=200)
                         if abs(mp.im(r)) < mp.mpf(10) ** (-30)]
                target = L.get(self.name).c2_mp
                tv = min((mp.re(r) for r in roots), key=lambda r: abs(r - target))
            vals = [mp.mpf(sp.N(wi.subs(t, sp.Float(str(tv), dps)), dps)) for wi in self.w]
        return tv, vals


def _shape(r2, d, order):
    return L.shape_factors(r2, d, order)


def moment_identity_failures(name: str, order: int):
    """List of (which, exponent) for which an identity of Sec. 4 fails."""
    lat = ExactLattice(name)
    d = lat.dim
    phis, chis = [], []
    for vec, w in zip(lat.v, lat.w):
        r2 = sp.Integer(sum(c * c for c in vec)) / t
        p, c = _shape(r2, d, order)
        phis.append(w * p)
        chis.append(w * c)
    fails = []
    for n in range(order + 1):
        for exps in itertools.product(range(n + 1), repeat=d):
            if sum(exps) != n:
                continue
            mono = [sp.Integer(1)] * len(lat.v)
            for i, vec in enumerate(lat.v):
                for a, e in enumerate(exps):
                    mono[i] *= sp.Integer(vec[a]) ** e
            if n == 0:
                tphi, tchi = 1, 1
            elif n == 2 and max(exps) == 2:
                tphi, tchi = t, 0
            else:
                tphi, tchi = 0, 0
            sphi = sum(p * m for p, m in zip(phis, mono))
            schi = sum(c * m for c, m in zip(chis, mono))
            if not lat.reduce(sphi - tphi):
                fails.append(("phi", exps))
            if not lat.reduce(schi - tchi):
                fails.append(("chi", exps))
    return fails
