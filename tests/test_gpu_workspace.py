"""GPU tests of caller-owned device state (lkp_problem_desc.workspace): a
handle whose state lives in a torch tensor gives the same bits as one that
allocated its own, allocates no device memory for it, and rejects workspaces
that are too small or misaligned."""
import sys

import numpy as np
import pytest
import torch

import paper_1504_05869_amd as lkp
from paper_1504_05869_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = [  # (lattice, order, shape, tau_lb, precision, population_sweep, in_place)
    ("D3Q111", 5, (13, 19, 37), 0.9, "f64", True, False),
    ("D2Q81", 5, (50, 70), 0.8, "f32_ir", True, True),
    ("D2Q25", 3, (37, 66), 1.3, "bf16dev_ir", True, False),
    ("D2Q169", 7, (41, 77), 1.0, "f32_ir", False, False),
    ("D3Q107", 5, (11, 21, 35), 1.0, "f32", False, False),
    ("D3Q111", 5, (13, 19, 37), 1.0, "f64", False, False),
]


def say(*a):
    print("[gpu-workspace]", *a, flush=True)
    sys.stdout.flush()


def _src(shape, seed):
    return W.zero_mean(np.random.default_rng(seed).standard_normal(shape))


def _run(s, lattice, order, tau, prec, pop, inp, **kw):
    with lkp.Problem(s, lattice, order, tau_lb=tau, precision=prec, population_sweep=pop,
                     in_place=inp, **kw) as p:
        if prec == "f32":   # plain FP32 stalls at its rounding floor: a fixed count
            rep = p.solve(tol_rel_l2=1e-300, max_sweeps=3000, check_every=50, raise_on_error=False)
        else:
            rep = p.solve(tol_rel_l2=1e-9, max_sweeps=400000, check_every=50)
        return p.phi_host(), rep, p.info()


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[4]}-tau{c[3]}" for c in CASES])
def test_workspace_state_equals_owned_state(case):
    """A solve to 1e-9 (plain FP32: 3000 sweeps; refinement cases included): Phi bitwise equal, same
    sweeps and refinement steps, same footprint."""
    lattice, order, shape, tau, prec, pop, inp = case
    s = _src(shape, 3)
    a, ra, ia = _run(s, lattice, order, tau, prec, pop, inp)
    b, rb, ib = _run(s, lattice, order, tau, prec, pop, inp, workspace=True)
    need = lkp.footprint_bytes(shape, lattice, order, tau_lb=tau, precision=prec, in_place=inp,
                               population_sweep=pop)
    say(case, "footprint", need, "sweeps", ra["sweeps"], rb["sweeps"], "outer", ra["outer"])
    assert ia["footprint_bytes"] == ib["footprint_bytes"] == need
    assert np.array_equal(a, b)
    assert ra["l2_change"] == rb["l2_change"] and ra["sweeps"] == rb["sweeps"]
    assert ra["outer"] == rb["outer"]


def test_workspace_in_a_larger_tensor_at_an_offset():
    """A slice of a larger byte tensor, 256-byte aligned, serves; the bytes
    around it are left as they were."""
    lattice, order, shape, tau = "D2Q81", 5, (40, 60), 0.9
    s = _src(shape, 5)
    need = lkp.footprint_bytes(shape, lattice, order, tau_lb=tau)
    big = torch.full((need + 4096,), 0xA5, dtype=torch.uint8, device="cuda")
    ws = big[1024:1024 + need]
    assert ws.data_ptr() % 256 == 0
    a, _, _ = _run(s, lattice, order, tau, "f64", True, False)
    b, _, _ = _run(s, lattice, order, tau, "f64", True, False, workspace=ws)
    assert np.array_equal(a, b)
    torch.cuda.synchronize()
    assert bool((big[:1024] == 0xA5).all()) and bool((big[1024 + need:] == 0xA5).all())


def test_workspace_too_small_or_misaligned_is_rejected():
    lattice, order, shape, tau = "D2Q25", 3, (32, 48), 0.8
    s = _src(shape, 6)
    need = lkp.footprint_bytes(shape, lattice, order, tau_lb=tau)
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(lkp.LkpError) as ei:
        lkp.Problem(s, lattice, order, tau_lb=tau, workspace=small)
    assert ei.value.name == "LKP_ERR_ARG"
    big = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(lkp.LkpError) as ei:
        lkp.Problem(s, lattice, order, tau_lb=tau, workspace=big[8:8 + need])
    assert ei.value.name == "LKP_ERR_ARG"
    say("too small and misaligned workspaces rejected")


def test_workspace_creation_allocates_no_device_memory():
    """With the workspace taken beforehand, creating and sweeping the handle
    leaves the device's free memory where it was (to 8 MiB, against a 250 MB
    state)."""
    lattice, order, shape, tau = "D3Q111", 5, (64, 64, 64), 0.9
    s = _src(shape, 7)
    with lkp.Problem(_src((8, 8, 8), 1), lattice, order, tau_lb=tau) as warm:
        warm.step(2)   # code objects and runtime state loaded once
    need = lkp.footprint_bytes(shape, lattice, order, tau_lb=tau)
    assert need > 2.5e8
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    p = lkp.Problem(s, lattice, order, tau_lb=tau, workspace=ws)
    p.step(3)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    phi = p.phi_host()
    p.close()
    say("free memory before / after creation", free0, free1, "state", need)
    assert free0 - free1 < 8 << 20
    assert np.isfinite(phi).all()
