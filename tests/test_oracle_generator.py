"""Pins of the velocity-set generator (quadrature conditions of Sec. 4)."""
import mpmath as mp
import numpy as np
import pytest

from oracle import exact as E
from oracle import generator as G
from oracle import lattice as L


def _found(name):
    sh = L.GENERATED_SHELLS[name]
    deg = L.generated_degree(name)
    sols = G.solve_subset(sh, G.classes(len(sh[0]), deg))
    assert len(sols) == 1
    t, W = sols[0]
    return G.Found(len(sh[0]), deg, sh, t, W, sum(len(G.orbit(r)) for r in sh))


def test_generator_reproduces_table_vector2():
    """Applied to the paper's ten D3Q111 shells, the generator's independent
    solve gives the oracle's c_s^2 and shell weights, and the printed digits."""
    shells = [b for b, _ in L.D3Q111_SHELLS]
    sols = G.solve_subset(shells, G.classes(3, 8))
    assert len(sols) == 1
    t, W = sols[0]
    lat = L.get("D3Q111")
    with mp.workdps(50):
        assert abs(t - lat.c2_mp) < mp.mpf(10) ** -40
        for (b, printed), w in zip(L.D3Q111_SHELLS, W):
            assert abs(w - lat.notes["shell_weights"][shells.index(b)]) < mp.mpf(10) ** -40
            p = mp.mpf(printed)
            digits = len(printed.split("e")[0].replace(".", "").lstrip("0"))
            unit = mp.mpf(10) ** (mp.floor(mp.log10(abs(p))) - digits + 1)
            assert abs(w - p) <= unit


def test_2d_search_finds_37_velocity_sets():
    res = G.search(2, 8, 3)
    assert {f.q for f in res} == {37} and len(res) == 4
    assert L.GENERATED_SHELLS["D2Q37"] in [f.reps for f in res]
    for f in res:  # every degree-9 2D set has the D3Q111 sound speed: 35 t^3 - 70 t^2 + 49 t - 12 = 0
        with mp.workdps(50):
            t = f.cs2
            assert abs(35 * t ** 3 - 70 * t ** 2 + 49 * t - 12) < mp.mpf(10) ** -40


@pytest.mark.parametrize("name", list(L.GENERATED_SHELLS))
def test_generated_sets_are_exact_quadratures(name):
    """Every monomial of degree <= D + 1 (odd ones included) has its Gaussian
    moment, with positive weights."""
    f = _found(name)
    v, w = f.velocities()
    assert all(x > 0 for x in w) and len(v) == f.q
    with mp.workdps(50):
        for n in range(f.degree + 2):
            for e in np.ndindex(*(n + 1,) * f.dim):
                if sum(e) != n:
                    continue
                m = mp.fsum(wi * mp.mpf(int(np.prod([int(x) ** a for x, a in zip(vec, e)])))
                            for vec, wi in zip(v, w))
                ref = L.gauss_moment(e, f.cs2)
                assert abs(m - ref) < mp.mpf(10) ** -35, (name, e)


@pytest.mark.parametrize("name,order", [("D2Q37", 5), ("D2Q77", 7), ("D3Q107", 5), ("D3Q103", 5)])
def test_generated_sets_satisfy_moment_identities(name, order):
    assert E.moment_identity_failures(name, order) == []


@pytest.mark.parametrize("name,order,tau,nk", [("D2Q37", 5, 0.65, 24), ("D2Q77", 7, 0.8, 24),
                                               ("D3Q107", 5, 0.65, 8)])
def test_generated_sets_are_stable_above_threshold(name, order, tau, nk):
    f = _found(name)
    for t in (tau, 1.0, 100.0):
        assert G.spectral_radius(f, order, t, nk) <= 1.0 + 1e-9


def test_d3q103_grows_at_order_5_only():
    """The smallest degree-9 3D set: stable at N = 3, but the checkerboard mode
    grows at N = 5 for every relaxation time (here 1, 10, 100)."""
    f = _found("D3Q103")
    assert G.spectral_radius(f, 3, 1.0, 4) <= 1.0 + 1e-9
    for t in (1.0, 10.0, 100.0):
        assert G.spectral_radius(f, 5, t, 2) > 1.0 + 1e-4   # k in {0, pi}^3


def test_3d_search_smallest_and_smallest_stable():
    """Components <= 3: the smallest degree-9 set has 103 velocities; requiring
    order-5 stability the smallest has 107, and the search also admits the
    paper's D3Q111 shells (checked by the Table vector2 test)."""
    plain = G.search(3, 8, 3)
    assert {f.q for f in plain} == {103}
    stable = G.search(3, 8, 3, require_stable_order=5)
    assert {f.q for f in stable} == {107}
    assert L.GENERATED_SHELLS["D3Q107"] in [f.reps for f in stable]


def test_planted_wrong_gaussian_moment_finds_nothing(monkeypatch):
    """Planted mistake: (a+1)!! instead of (a-1)!! in the target moments; the
    D2Q37 shells then admit no set with positive weights."""
    def wrong(e, t):
        m = 1
        for a in e:
            m *= G._dfact(a + 1)
        return m * t ** (sum(e) // 2)
    monkeypatch.setattr(G, "gauss_moment", wrong)
    assert G.solve_subset(L.GENERATED_SHELLS["D2Q37"], G.classes(2, 8)) == []


# 22 shells (components up to 6) found by a randomized search over shell subsets
SHELLS_3D_DEG12 = [(0, 0, 0), (1, 1, 1), (2, 2, 2), (6, 1, 1), (3, 3, 3), (3, 0, 0), (4, 1, 1),
                   (6, 0, 0), (5, 3, 1), (6, 3, 2), (2, 2, 0), (5, 1, 1), (3, 1, 1), (5, 5, 5),
                   (6, 5, 2), (3, 1, 0), (4, 3, 0), (4, 3, 2), (3, 2, 1), (6, 3, 0), (4, 2, 0),
                   (2, 0, 0)]


def test_3d_degree12_set_exists_but_order7_grows():
    """A cubic set exact for every monomial of degree <= 13 (the N = 7
    conditions) with positive weights: 495 velocities, one admissible c_s^2.
    Its N = 7 scheme has a growing mode (unlike N = 5 on the same set)."""
    sols = G.solve_subset(SHELLS_3D_DEG12, G.classes(3, 12))
    assert len(sols) == 1
    t, W = sols[0]
    assert all(w > 0 for w in W)
    f = G.Found(3, 12, SHELLS_3D_DEG12, t, W, sum(len(G.orbit(r)) for r in SHELLS_3D_DEG12))
    assert f.q == 495
    assert abs(float(t) - 2.18400454768877) < 1e-12
    assert G.spectral_radius(f, 7, 1.0, nk=4) > 1.03
    assert G.spectral_radius(f, 5, 1.0, nk=4) <= 1.0 + 1e-9
