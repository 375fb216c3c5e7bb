"""Pins of the oracle's lattice constants against the paper and exact mathematics."""
import json
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import exact as E
from oracle import lattice as L

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
ALL = ["D1Q5", "D1Q9", "D1Q13", "D2Q5", "D2Q9", "D2Q25", "D2Q81", "D2Q169", "D3Q111"]

# degree through which each set must integrate Gaussian moments exactly
EXACT_DEGREE = {"D1Q5": 6, "D1Q9": 10, "D1Q13": 12, "D2Q25": 6, "D2Q81": 10,
                "D2Q169": 12, "D3Q111": 8, "D2Q5": 2, "D2Q9": 4}


def last_digit_unit(printed):
    """One unit in the last printed digit (rounding or truncation stays below it)."""
    mant, _, exp = printed.partition("e")
    decimals = len(mant.split(".")[1]) if "." in mant else 0
    return mp.mpf(10) ** (int(exp or 0) - decimals)


def _monomials(dim, deg):
    import itertools
    for e in itertools.product(range(deg + 1), repeat=dim):
        if sum(e) <= deg:
            yield e


@pytest.mark.parametrize("name", ALL)
def test_quadrature_exactness(name):
    """Eq. (quadrature)/(quad3): the discrete weights reproduce the Gaussian moments."""
    lat = L.get(name)
    deg = EXACT_DEGREE[name]
    with mp.workdps(50):
        for e in _monomials(lat.dim, deg):
            if lat.dim >= 2 and max(e) > (deg if name not in ("D2Q5",) else 2):
                continue
            # tensor-product sets are exact per axis, D3Q111 in total degree
            if lat.dim == 2 and name in ("D2Q25", "D2Q81", "D2Q169") and sum(e) > deg:
                continue
            m = mp.fsum(w * mp.fprod(mp.mpf(int(c)) ** k for c, k in zip(v, e))
                        for v, w in zip(lat.v, lat.w_mp))
            ref = L.gauss_moment(e, lat.c2_mp)
            assert abs(m - ref) < mp.mpf(10) ** -40, (name, e, m, ref)


def test_tensor_sets_exact_beyond_total_degree():
    """Tensor products are exact for every x^a y^b with a, b within the 1D degree."""
    lat = L.get("D2Q169")
    with mp.workdps(50):
        for a, b in [(12, 12), (10, 6), (12, 2)]:
            m = mp.fsum(w * mp.mpf(int(v[0])) ** a * mp.mpf(int(v[1])) ** b
                        for v, w in zip(lat.v, lat.w_mp))
            assert abs(m - L.gauss_moment((a, b), lat.c2_mp)) < mp.mpf(10) ** -35


@pytest.mark.parametrize("name,key", [("D1Q5", "appendix_D1Q5"), ("D1Q9", "appendix_D1Q9"),
                                      ("D1Q13", "appendix_D1Q13")])
def test_1d_weights_match_appendix(name, key):
    g = GOLD[key]
    lat = L.get(name)
    assert [int(x) for x in lat.v[:, 0]] == g["speeds"]
    with mp.workdps(50):
        for w, printed in zip(lat.w_mp, g["weights"]):
            p = mp.mpf(printed)
            assert abs(w - p) <= last_digit_unit(printed), (name, w, printed)


def test_sound_speeds_match_appendix():
    with mp.workdps(50):
        assert abs(L.get("D1Q5").c2_mp - (1 - mp.sqrt(mp.mpf(2) / 5))) < mp.mpf(10) ** -45
        # the Appendix values labelled c_s^2 for N=5 and N=7 are c_s
        c9 = mp.sqrt(L.get("D1Q9").c2_mp)
        assert abs(c9 - mp.mpf(GOLD["appendix_D1Q9"]["printed_cs2_label_value"])) < 1e-15
        c13 = mp.sqrt(L.get("D1Q13").c2_mp)
        assert abs(c13 - mp.mpf(GOLD["appendix_D1Q13"]["printed_cs2_label_value"])) < 1e-30
    # Sec. 4 quotes "about 0.4" for N=3 (c_s^2 = 0.37) and "nearly 1.2" for
    # N=7 (c_s = 1.15): the text mixes c_s^2 and c_s as the Appendix does
    assert 0.35 < L.get("D1Q5").c2 < 0.4
    assert 1.1 < float(mp.sqrt(L.get("D1Q13").c2_mp)) < 1.2


def test_appendix_weights_give_printed_cs_squared():
    """Reading the N=5/N=7 'c_s^2' entries as c_s: the printed weights' own
    second moment equals the printed value squared."""
    for key in ("appendix_D1Q9", "appendix_D1Q13"):
        g = GOLD[key]
        with mp.workdps(40):
            m2 = mp.fsum(mp.mpf(w) * v * v for w, v in zip(g["weights"], g["speeds"]))
            c = mp.mpf(g["printed_cs2_label_value"])
            assert abs(m2 - c * c) < 1e-15
            assert abs(m2 - c) > 0.1


def test_d3q111_matches_table_vector2():
    g = GOLD["table_vector2_D3Q111"]
    lat = L.get("D3Q111")
    assert lat.Q == 111
    weights = lat.notes["shell_weights"]
    for (base, printed, mult), w in zip(g["shells"], weights):
        assert len(L._orbit(tuple(base))) == mult
        with mp.workdps(50):
            assert abs(w - mp.mpf(printed)) <= last_digit_unit(printed), (base, w, printed)
    assert sum(m for _, _, m in g["shells"]) == 111


def test_d3q111_sound_speed_is_cubic_root():
    """The admissible c_s^2 derived in exact arithmetic (oracle.exact) is a
    root of 35 t^3 - 70 t^2 + 49 t - 12 and equals the numeric solve."""
    ex = E.ExactLattice("D3Q111")
    assert [int(c) for c in ex.modulus.all_coeffs()] == [35, -70, 49, -12]
    with mp.workdps(50):
        assert abs(mp.polyval([35, -70, 49, -12], L.get("D3Q111").c2_mp)) < mp.mpf(10) ** -45


@pytest.mark.parametrize("name", ["D1Q5", "D1Q9", "D1Q13", "D2Q25", "D3Q111"])
def test_exact_weights_equal_numeric(name):
    ex = E.ExactLattice(name)
    tv, vals = ex.weight_values(50)
    lat = L.get(name)
    with mp.workdps(50):
        assert abs(tv - lat.c2_mp) < mp.mpf(10) ** -40
        for a, b in zip(vals, lat.w_mp):
            assert abs(a - b) < mp.mpf(10) ** -40


CASES = [("D1Q5", 1), ("D1Q5", 3), ("D1Q9", 1), ("D1Q9", 3), ("D1Q9", 5), ("D1Q13", 7),
         ("D2Q5", 1), ("D2Q9", 1), ("D2Q9", 3), ("D2Q25", 1), ("D2Q25", 3),
         ("D2Q81", 5), ("D3Q111", 5)]


@pytest.mark.parametrize("name,order", CASES)
def test_moment_identities_exact(name, order):
    """Sec. 4: Pi(0)=Phi, Pi(1)=0, Pi(2)=c_s^2 Phi, Pi(n>2)=0, S(0)=S, S(n>0)=0
    up to order N, in exact arithmetic."""
    assert E.moment_identity_failures(name, order) == []


@pytest.mark.slow
def test_moment_identities_exact_d2q169():
    assert E.moment_identity_failures("D2Q169", 7) == []


@pytest.mark.parametrize("name,order", [("D1Q5", 5), ("D2Q5", 3), ("D2Q25", 5), ("D1Q9", 7)])
def test_identities_fail_beyond_lattice_order(name, order):
    """Negative control: a set too small for the order violates the identities."""
    assert E.moment_identity_failures(name, order) != []


def test_printed_he4_typo_breaks_identities(monkeypatch):
    """Planted mistake in the oracle: taking the He4 numerator literally as
    3 c_s^2 - 6 c_s^2 v^2 + v^4 (as printed in Eq. omega:eq) breaks Pi(4) = 0."""
    orig = L.radial_hermite

    def typo(r2, d):
        R2, R4, R6 = orig(r2, d)
        # 3 c^2 / c^4 = 3 / c^2 in place of 3: r2 carries 1/t, so 3/t = 3 * r2 / v^2;
        # use the 1D form directly with t symbolic
        from oracle.exact import t
        return R2, R4 - 3 + 3 / t, R6
    monkeypatch.setattr(L, "radial_hermite", typo)
    assert E.moment_identity_failures("D1Q13", 7) != []


def test_paper_formulas_equal_radial_form():
    """Eq. omega:eq / chi:eq (1D, N=7, with 3 c_s^4) and Eq. omega:eq3 /
    chi:eq3 (3D, N=5) written out as printed agree with the radial form."""
    with mp.workdps(40):
        lat = L.get("D1Q13")
        c2 = lat.c2_mp
        phi, chi = L.coefficients_mp(lat, 7)
        for v, w, p, c in zip(lat.v[:, 0], lat.w_mp, phi, chi):
            v = mp.mpf(int(v))
            he4 = (3 * c2 ** 2 - 6 * c2 * v ** 2 + v ** 4) / (8 * c2 ** 2)
            he6 = (15 * c2 ** 3 - 45 * c2 ** 2 * v ** 2 + 15 * c2 * v ** 4 - v ** 6)
            p_paper = w * (1 - he4 - he6 / (24 * c2 ** 3))
            c_paper = w * (1 + (1 - v ** 2 / c2) / 2 + he4 + he6 / (48 * c2 ** 3))
            assert abs(p - p_paper) < 1e-35 and abs(c - c_paper) < 1e-35
        lat = L.get("D3Q111")
        c2 = lat.c2_mp
        phi, chi = L.coefficients_mp(lat, 5)
        for v, w, p, c in zip(lat.v, lat.w_mp, phi, chi):
            v2 = mp.mpf(int(sum(int(x) ** 2 for x in v)))
            q = (15 * c2 ** 2 - 10 * c2 * v2 + v2 ** 2) / (8 * c2 ** 2)
            assert abs(p - w * (1 - q)) < 1e-35
            assert abs(c - w * (1 + (3 - v2 / c2) / 2 + q)) < 1e-35


def test_coefficient_sums_and_symmetry():
    for name, order in CASES:
        lat = L.get(name)
        phi, chi = L.coefficients(lat, order)
        assert abs(phi.sum() - 1) < 1e-14 and abs(chi.sum() - 1) < 1e-14
        # closed under v -> -v with equal coefficients
        idx = {tuple(v): i for i, v in enumerate(lat.v.tolist())}
        for i, v in enumerate(lat.v.tolist()):
            j = idx[tuple(-x for x in v)]
            assert phi[i] == phi[j] and chi[i] == chi[j]


def test_order_above_lattice_maximum_rejected():
    with pytest.raises(ValueError):
        L.coefficients(L.get("D2Q81"), 7)


def test_knudsen_mapping():
    lat = L.get("D2Q81")
    tau = L.tau_from_knudsen(0.1, lat, 1024)
    assert abs(np.sqrt(lat.c2) * (tau - 0.5) / 1024 - 0.1) < 1e-14
