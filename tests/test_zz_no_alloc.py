"""GPU test of lkp_residual_noalloc (the residual sweep of lkp_residual with no
device allocation) through the C ABI: its norms equal lkp_residual's on the
same state, and its Phi and residual populations equal the oracle's."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import paper_1504_05869_amd as lkp
from paper_1504_05869_amd import _lib
from paper_1504_05869_amd import workloads as W
from oracle import lattice as OL
from oracle import sweep as SW

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-noalloc]", *a, flush=True)
    sys.stdout.flush()


def _perm(lattice):
    """perm[i] = oracle index of the product's velocity i."""
    info = lkp.lattice_info(lattice, 1)
    idx = {tuple(int(c) for c in v): i for i, v in enumerate(OL.get(lattice).v3())}
    return np.array([idx[tuple(int(c) for c in v)] for v in info["v"]])


def _grid(shape):
    return (ctypes.c_int64 * 3)(*(list(shape)[::-1] + [1] * (3 - len(shape))))


def _noalloc(lattice, order, shape, tau, f_dev, S_dev, phi_prev_dev):
    Q = f_dev.shape[0]
    phi_out = torch.empty(shape, dtype=torch.float64, device="cuda")
    r_out = torch.empty((Q,) + tuple(shape), dtype=torch.float32, device="cuda")
    norms = torch.full((6,), float("nan"), dtype=torch.float64, device="cuda")
    st = _lib.load().lkp_residual_noalloc(
        _lib.LATTICES[lattice], order, _grid(shape), tau, f_dev.data_ptr(), S_dev.data_ptr(),
        phi_prev_dev.data_ptr(), phi_out.data_ptr(), r_out.data_ptr(), norms.data_ptr(),
        torch.cuda.current_stream().cuda_stream)
    _lib.check(st, "lkp_residual_noalloc")
    torch.cuda.synchronize()
    return phi_out.cpu().numpy(), r_out.cpu().numpy(), norms.cpu().numpy()


def _case(lattice, order, shape, tau, seed):
    rng = np.random.default_rng(seed)
    s = W.zero_mean(rng.standard_normal(shape))
    Q = lkp.lattice_info(lattice)["Q"]
    f0 = rng.standard_normal((Q,) + tuple(shape))           # product velocity order
    # the existing entry point: a handle, two sweeps, lkp_residual
    with lkp.Problem(s, lattice, order, tau_lb=tau) as p:
        p.set_populations(f0)
        p.step(2)
        rep = p.residual()
        phi2 = p.phi()                                         # Phi of sweep 2 (device)
        f2 = p.populations()                                   # f* after sweep 2 (host)
    info = lkp.lattice_info(lattice, order)
    S = s * (info["cs2"] * (tau - 0.5))                       # the scaled source
    f_dev = torch.from_numpy(f2).cuda()
    S_dev = torch.from_numpy(S).cuda()
    phi3, r, nr = _noalloc(lattice, order, shape, tau, f_dev, S_dev, phi2)
    # norms: the same quantities as lkp_residual's report
    ours = {"max_change": nr[0], "l2_change": np.sqrt(nr[1]), "phi_l2": np.sqrt(nr[2]),
            "mass": nr[3], "pop_residual_l2": np.sqrt(nr[5])}
    bitwise = all(ours[k] == rep[k] for k in ours)
    say(lattice, shape, "norms bitwise equal to lkp_residual:", bitwise, ours, rep)
    assert nr[4] == 0
    for k, v in ours.items():
        scale = max(abs(rep[k]), rep["phi_l2"] * 1e-3)
        assert abs(v - rep[k]) <= 1e-13 * scale, k
    # Phi and r against the oracle (three sweeps from f0)
    pm = _perm(lattice)
    inv = np.argsort(pm)
    prob = SW.Problem(lattice, order, tau, s)
    f0_o = f0[inv]                                              # oracle velocity order
    _, f2_o = SW.run(prob, 2, f0_o)
    phi3_o, f3_o = SW.run(prob, 1, f2_o)
    e_phi = np.linalg.norm(phi3 - phi3_o) / np.linalg.norm(phi3_o)
    r_o = (f3_o - f2_o)[pm]
    e_r = np.linalg.norm(r - r_o) / np.linalg.norm(r_o)
    say(lattice, shape, "Phi vs oracle", e_phi, "r vs oracle (FP32 storage)", e_r)
    assert e_phi <= 1e-13
    assert e_r <= 1e-6


def test_noalloc_residual_equals_lkp_residual_two_calls():
    """Two calls in a row, the second on a smaller grid (the shared scratch
    keeps the first call's partials beyond the second's blocks)."""
    _case("D3Q111", 5, (40, 44, 48), 1.7, 1)
    _case("D3Q111", 5, (12, 10, 16), 2.3, 2)


def test_noalloc_residual_other_sets():
    _case("D2Q169", 7, (40, 52), 3.0, 3)      # four velocity groups
    _case("D2Q81", 5, (33, 29), 1.4, 4)


def test_noalloc_rejects_oversize_grid_without_launching():
    """Beyond 2^24 cells the fixed scratch cannot hold the partials: the call
    fails on the host, before anything is enqueued."""
    lib = _lib.load()
    t = torch.zeros(8, dtype=torch.float64, device="cuda")
    p = t.data_ptr()
    st = lib.lkp_residual_noalloc(_lib.LATTICES["D3Q111"], 5, _grid((512, 512, 512)), 2.0,
                                  p, p, p, p, None, p, None)
    assert _lib.STATUS[st] == "LKP_ERR_ARG"
    st = lib.lkp_residual_noalloc(_lib.LATTICES["D3Q111"], 7, _grid((8, 8, 8)), 2.0,
                                  p, p, p, p, None, p, None)
    assert _lib.STATUS[st] == "LKP_ERR_LATTICE_ORDER"
    torch.cuda.synchronize()
    assert torch.all(t == 0)
