"""Benchmark of the lattice-kinetic Poisson sweep on one MI355X.

Headline workload (one GPU): periodic 512^3 grid, higher-order scheme at order
N = 5 on D3Q111 (Appendix A, Table vector2), Kn = 0.3 (tau_lb = 184.36),
source = 4096 point-like Gaussians of width 1 cell with amplitudes +-U(1,10)
at seeded uniform positions, mean removed; FP64 populations in two buffers
(238 GB of the 288 GB of HBM).

A step is one pass of the solver's hot path: one chunk of --chunk sweeps
(fused pull-stream / moment / collide+source), the FP64 convergence
reductions on the last two sweeps, the read-back of the norms and the host's
stopping decision against rel-L2 1e-10 (a real decision: the convergence
history carries across steps).  Inputs are resident in HBM before timing
starts.

Printed: one JSON line with GLUPS (cell updates per second; one update moves
all Q populations of a cell), the roofline of the sweep kernel from HIP events
on the solver's stream over the timed region, the oracle's CPU throughput on a
bounded sample, and extra measurements (other sets, orders and precisions,
time-to-solution with each answer's error against the oracle's exact fixed
point, serving).
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
ORDERS = {1: "D2Q25", 3: "D2Q25", 5: "D2Q81", 7: "D2Q169"}
# the headline problem: 512^3 D3Q111 N = 5, Kn = 0.3, 4096 point-like Gaussians
C5 = {"shape": (512, 512, 512), "lattice": "D3Q111", "order": 5, "knudsen": 0.3,
      "kind": "stiff3d", "seed": 5120}


def bytes_per_cell(Q: int, precision: str) -> int:
    """Algorithmic HBM bytes of one sweep per cell (pull, two buffers):
    read Q populations + write Q populations + read S."""
    b = 8 if precision == "f64" else 4
    return 2 * b * Q + b


def r_q(lkp, lattice: str) -> int:
    return int(lkp.lattice_info(lattice)["Q"])


def sweep_rate(lkp, torch, s, lattice, order, precision, knudsen=None, tau_lb=None,
               sweeps=200, chunks=1, population_sweep=False, in_place=False, drift=None):
    """Average duration of one sweep (HIP events on the solver's stream), timed
    after about 0.2 s of untimed sweeps on the same problem, so that the GPU's
    clocks have settled: a few hundred sweeps of a small grid otherwise run
    while the clocks are still rising."""
    with lkp.Problem(s, lattice, order, knudsen=knudsen, tau_lb=tau_lb, precision=precision,
                     population_sweep=population_sweep, in_place=in_place, drift=drift) as p:
        p.step(2)
        p.sync()
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 0.2:
            p.step(sweeps)
            p.sync()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(chunks):
            p.step(sweeps)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / (sweeps * chunks)
        info = p.info()
    n = int(np.prod(s.shape))
    bpc = bytes_per_cell(info["Q"], precision)
    return {"lattice": lattice, "order": order, "precision": precision,
            "ms_per_sweep": ms, "glups": n / (ms * 1e-3) / 1e9,
            "gbs": n * bpc / (ms * 1e-3) / 1e9,
            "frac_hbm": n * bpc / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "velocity_groups": info["velocity_groups"], "tau_lb": info["tau_lb"],
            "stencil_tile": info["stencil_tile"], "stencil_remap": info["stencil_remap"],
            "form": "stencil (tau_lb=1)" if info["scalar_stencil"] else
                    ("population sweep, in place" if in_place else "population sweep")}


KERNEL_SOURCES = ["paper_1504_05869_amd/csrc/sweep_impl.hpp", "paper_1504_05869_amd/csrc/lattices.hpp",
                  "paper_1504_05869_amd/csrc/kernels.hpp", "paper_1504_05869_amd/csrc/device_common.hpp"]


def measured_traffic(tag: str):
    """HBM bytes per launch from the committed counter summary, or None when the
    kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{tag}.traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec.get("kernel_source_sha256"):
        return None
    return int(round(rec["traffic_bytes"]))


def paper_context(eps=1e-3):
    """The paper's own comparison of orders, quoted as context: time to error
    eps from its 1D fits (Table 1: throughput xi_N, steps scale b_N, error
    fit a_N L^-alpha_N) through Eq. TEPS, t_N = (b_N / xi_N) (a_N / eps)^(3 / alpha_N),
    on hardware the paper does not state."""
    fits = {1: (26.2e6, 10.98, 1.645, 1), 3: (21.4e6, 10.98, 1.645, 1),
            5: (5.44e6, 5.46, 33.11, 3), 7: (5.76e6, 3.23, 992.3, 5)}
    t = {n: b / xi * (a / eps) ** (3.0 / al) for n, (xi, b, a, al) in fits.items()}
    return {"what": "standard LB (N=1) vs higher order, time to error 1e-3 in 1D, from the "
                    "paper's Table 1 fits and Eq. TEPS (hardware and precision unstated; context "
                    "only, not a measurement here)",
            "seconds_by_order": {str(n): float(f"{v:.4g}") for n, v in t.items()},
            "speedup_N1_over_N7": float(f"{t[1] / t[7]:.3g}")}


def true_rel_l2(phi: np.ndarray, ref: np.ndarray) -> float:
    """||phi - ref||_2 / ||ref||_2 (no mean removed: a mass drift counts)."""
    return float(np.linalg.norm((phi - ref).ravel()) / np.linalg.norm(ref.ravel()))


def oracle_fixed_point(lattice, order, s, tau_lb=None, knudsen=None):
    """The oracle's exact fixed point (spectral, FP64) of a problem; tau_lb
    from Kn with the oracle's own mapping.  Reference generation, outside every
    timed region."""
    from oracle import lattice as OL
    from oracle import spectral as SP
    if tau_lb is None:
        tau_lb = OL.tau_from_knudsen(knudsen, OL.get(lattice), min(s.shape))
    return SP.fixed_point_large(lattice, order, tau_lb, s)


def timed_solve(lkp, torch, s, lattice, order, precision, tol, ref=None, check_every=100,
                chunk=0, label="", max_seconds=0.0, **kw) -> dict:
    """Solve to estimated rel-L2 `tol`; wall time, sweeps, the solver's own
    estimate and, with `ref`, the true error against the oracle's fixed point.
    chunk > 0: consecutive lkp_solve calls of at most `chunk` sweeps (a resumed
    call keeps the convergence history, a stopped refinement its partial
    correction), one progress line each; max_seconds > 0 then also caps the
    wall time (the report says whether the tolerance was reached)."""
    with lkp.Problem(s, lattice, order, precision=precision, **kw) as q:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sweeps, outer = 0, 0
        while True:
            rep = q.solve(tol_rel_l2=tol, check_every=check_every,
                          max_sweeps=chunk if chunk > 0 else 4_000_000, raise_on_error=False)
            sweeps += rep["sweeps"]
            outer = rep["outer"] if precision in ("f64", "f32") else outer + rep["outer"]
            if chunk <= 0 or rep["status"] == 0 or sweeps >= 4_000_000:
                break
            if max_seconds > 0 and time.perf_counter() - t1 > max_seconds:
                break
            say(f"{label} {precision}: {sweeps} sweeps {time.perf_counter() - t1:.0f} s "
                f"est {rep['est_rel_err']:.3e}")
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        out = {"precision": precision, "tol_rel_l2": tol, "seconds": round(el, 4),
               "sweeps": sweeps, "outer": outer, "status": rep["status"],
               "converged": rep["status"] == 0, "est_rel_err": rep["est_rel_err"]}
        if ref is not None:
            out["true_rel_l2"] = true_rel_l2(q.phi_host(), ref)
    return out


def cpu_baseline(s, lattice, order, tau, seconds=15.0, note=""):
    """Oracle C sweep (FP64, OpenMP) on a grid for a bounded time."""
    from oracle import sweep as SW
    prob = SW.Problem(lattice, order, tau, s)
    a = prob.zero_state()
    b = np.empty_like(a)
    Phi = np.empty(s.shape)
    SW.sweep_c(prob, a, b, Phi)                 # warm (page in)
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < seconds or k < 2:
        SW.sweep_c(prob, a, b, Phi)
        a, b = b, a
        k += 1
    dt = time.perf_counter() - t0
    grid = "x".join(str(n) for n in s.shape[::-1])
    return {"value": s.size * k / dt / 1e9, "unit": "GLUPS", "cores": SW.threads(),
            "kind": "oracle",
            "sample": f"{k} full sweeps of the {grid} {lattice} N={order} tau_lb={tau:.2f} FP64 "
                      f"grid in {dt:.1f} s{note}"}


def headline(lkp, torch, args) -> dict:
    """K timed steps of the 512^3 D3Q111 FP64 sweep (see the module docstring)."""
    from paper_1504_05869_amd import workloads as W
    shape, lattice, order, kn = C5["shape"], C5["lattice"], C5["order"], C5["knudsen"]
    s = W.poisson_source(C5["kind"], shape, seed=C5["seed"])
    n = s.size
    p = lkp.Problem(s, lattice, order, knudsen=kn, precision="f64")
    del s
    info = p.info()
    Q = info["Q"]
    say(f"headline: {info['n']} {lattice} N={order} tau_lb={info['tau_lb']:.4f} FP64, "
        f"{info['footprint_bytes'] / 1e9:.1f} GB resident, split P={info['velocity_groups']}")

    def step():
        # one chunk with its convergence check against the 1e-10 target; the
        # contraction history carries over, so each check is a real decision
        return p.solve(tol_rel_l2=1e-10, max_sweeps=args.chunk, check_every=args.chunk,
                       use_graph=True, raise_on_error=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    say(f"headline: {args.warmup} warmup steps done, timing {args.steps} steps")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    sweeps, last = 0, None
    for _ in range(args.steps):
        last = step()
        sweeps += last["sweeps"]
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # every launch of the timed region on the solver's stream (torch's current
    # stream): the sweeps, their norm finishes; divided over the sweeps
    ms_sweep = e0.elapsed_time(e1) / sweeps
    p.close()
    glups = n * sweeps / wall / 1e9
    bpc = bytes_per_cell(Q, "f64")
    achieved = n * bpc / (ms_sweep * 1e-3) / 1e9
    return {
        "metric": "GLUPS (lattice cell updates per second, all Q populations per update)",
        "value": round(glups, 4),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D periodic 512^3 Poisson, D3Q111 N=5, Kn=0.3 "
                               f"(tau_lb={info['tau_lb']:.4f}), 4096 Gaussians sigma=1, amplitudes "
                               "+-U(1,10), zero mean; FP64 populations, two buffers",
                   "grid": list(shape), "lattice": lattice, "order": order, "knudsen": kn,
                   "sweeps_per_step": args.chunk, "velocity_groups": info["velocity_groups"],
                   "footprint_gb": round(info["footprint_bytes"] / 1e9, 1)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("k_sweep_d3q111_f64_512cubed"),
                     "kernel": "k_sweep (D3Q111, FP64, two buffers)",
                     "bytes_per_launch": n * bpc, "ms_per_launch": round(ms_sweep, 5)},
        "paper_context": paper_context(),
        "last_check": {"est_rel_err": last["est_rel_err"], "rate": last["rate"],
                       "total_sweeps": last["total_sweeps"]},
    }


def stiff_512(lkp, torch, tol: float, chunk: int, minutes: float) -> dict:
    """The headline problem solved to estimated rel-L2 `tol`: FP32 sweeps +
    FP64 refinement (in place: 242 GB) against the plain FP64 sweep (two
    buffers: 242 GB).  The solve runs as consecutive lkp_solve calls of
    `chunk` sweeps (a resumed call keeps the convergence history; a refinement
    stopped by max_sweeps keeps its partial correction), one progress line per
    call on stderr.  Each answer is compared with the oracle's exact fixed
    point (spectral, FP64, computed on the host after the timed solves).  A
    solve still short of `tol` after `minutes` of wall time reports its reached
    error and a time extrapolated from its rate (labelled as such)."""
    from paper_1504_05869_amd import workloads as W
    shape = C5["shape"]
    t0 = time.perf_counter()
    s = W.poisson_source(C5["kind"], shape, seed=C5["seed"])
    gen_s = time.perf_counter() - t0
    out = {"workload": "512^3 D3Q111 N=5 Kn=0.3, 4096 Gaussians sigma=1, amplitudes +-U(1,10), zero mean",
           "tol_rel_l2": tol, "source_generation_s": round(gen_s, 1), "runs": []}
    phis = []
    for prec, in_place in (("f32_ir", True), ("f64", False)):
        with lkp.Problem(s, "D3Q111", 5, knudsen=C5["knudsen"], precision=prec, in_place=in_place) as q:
            info = q.info()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sweeps, outer, rep = 0, 0, None
            while True:
                rep = q.solve(tol_rel_l2=tol, check_every=200, max_sweeps=chunk, raise_on_error=False)
                sweeps += rep["sweeps"]
                outer = rep["outer"] if prec == "f64" else outer + rep["outer"]
                el = time.perf_counter() - t1
                say(f"[c5] {prec} in_place={in_place} {sweeps} sweeps {el:.0f} s est "
                    f"{rep['est_rel_err']:.3e} status {rep['status']}")
                if rep["status"] == 0 or el > 60 * minutes:
                    break
            torch.cuda.synchronize()
            el = time.perf_counter() - t1
            run = {"precision": prec, "in_place": in_place, "footprint_gb": round(info["footprint_bytes"] / 1e9, 1),
                   "converged": rep["status"] == 0, "seconds": round(el, 1), "sweeps": sweeps,
                   "outer": outer, "est_rel_err": rep["est_rel_err"], "rate": rep["rate"],
                   "ms_per_sweep": round(el / max(sweeps, 1) * 1e3, 2)}
            if rep["status"] != 0 and 0 < rep["rate"] < 1 and rep["est_rel_err"] > tol:
                import math
                more = math.log(tol / rep["est_rel_err"]) / math.log(rep["rate"])
                run["extrapolated_seconds"] = round(el + more * el / max(sweeps, 1), 1)
            phis.append(q.phi_host())
            out["runs"].append(run)
    t2 = time.perf_counter()
    ref = oracle_fixed_point("D3Q111", 5, s, knudsen=C5["knudsen"])
    out["reference_generation_s"] = round(time.perf_counter() - t2, 1)
    for run, phi in zip(out["runs"], phis):
        run["true_rel_l2"] = true_rel_l2(phi, ref)
    return out


def serving_run(n_requests: int, rate: float, full_sizes: bool = False) -> dict:
    """Serving stream: continuous batching (FP32 + refinement, states in
    workspaces from torch's caching allocator; once more with per-problem
    device allocations) against the same trace solved one at a time in FP64,
    all to estimated rel-L2 1e-6.  Every
    answer is read back at retirement and compared afterwards with the
    oracle's exact fixed point.  The default size mix is scaled down so that
    the run takes seconds; full_sizes draws from {128..2048}^2 and
    {64,128,256}^3 with a 240 GiB HBM budget."""
    from paper_1504_05869_amd import serve
    if full_sizes:
        s2 = tuple((n, n) for n in (128, 256, 512, 1024, 2048))
        s3 = tuple((n, n, n) for n in (64, 128, 256))
        budget = 240 << 30
    else:
        s2 = ((64, 64), (128, 128), (256, 256), (512, 512))
        s3 = ((32, 32, 32), (48, 48, 48), (64, 64, 64))
        budget = 64 << 30
    reqs = serve.make_stream(n_requests, rate=rate, seed=2024, sizes2d=s2, sizes3d=s3)
    # requests arrive carrying their source fields (synthesised here, untimed)
    serve.attach_sources(reqs)

    def prog(msg):
        if full_sizes:
            say(f"[serving] {msg}")

    # warm-up on the first requests (code objects, split tuning per class), so
    # that neither batched leg pays for it
    serve.Server(serve.GpuBackend("f32_ir", workspace=False), hbm_budget=budget,
                 sweeps_per_tick=50, tol=1e-6).run(reqs[:8])
    srv = serve.Server(serve.GpuBackend("f32_ir", keep_phi=True), hbm_budget=budget,
                       sweeps_per_tick=50, tol=1e-6, progress=prog)
    res, summ = srv.run(reqs)
    # the same batched leg with every problem allocating its own device state
    # (scaled sizes only: at full sizes allocation is a small share of a solve)
    osum = None
    if not full_sizes:
        own = serve.Server(serve.GpuBackend("f32_ir", workspace=False), hbm_budget=budget,
                           sweeps_per_tick=50, tol=1e-6, progress=prog)
        _, osum = own.run(reqs)
    base, bsum = serve.run_one_at_a_time(reqs, "f64", tol=1e-6, check_every=50, keep_phi=True,
                                         progress=prog)
    # latency at an offered load below capacity: the same requests arriving at
    # 0.8 x the batched leg's measured problems/s (arrival times scaled), both
    # ways of serving them
    load = 0.8 * summ["problems_per_s"]
    scale = rate / load
    slow = [dataclasses.replace(r, arrival=r.arrival * scale) for r in reqs]
    _, lsum = serve.Server(serve.GpuBackend("f32_ir"), hbm_budget=budget, sweeps_per_tick=50,
                           tol=1e-6, progress=prog).run(slow)
    _, lbase = serve.run_one_at_a_time(slow, "f64", tol=1e-6, check_every=50, progress=prog)
    # true errors against the oracle (after both legs; not timed)
    errs = {"batched": [], "one_at_a_time": []}
    by_rid = {r.rid: r for r in reqs}
    for leg, results in (("batched", res), ("one_at_a_time", base)):
        for r in results:
            if r.phi is None:
                continue
            q = by_rid[r.rid]
            ref = oracle_fixed_point(q.lattice, q.order, q.source_field(), knudsen=q.knudsen)
            errs[leg].append(true_rel_l2(r.phi, ref))
            r.phi = None
    keys = ("completed", "problems_per_s", "p50_latency_s", "p99_latency_s", "makespan_s",
            "sweeps_total")
    sizes = ("{128,256,512,1024,2048}^2 and 3D D3Q111 N=5 {64,128,256}^3" if full_sizes else
             "{64,128,256,512}^2 and 3D D3Q111 N=5 {32,48,64}^3")

    def err_stats(v):
        return {"max": max(v), "median": float(np.median(v)), "count": len(v)} if v else None

    return {"stream": f"{n_requests} requests, Poisson arrivals at {rate}/s, 2D D2Q81 N=5 "
                      f"{sizes}, Kn~U(0.05,0.5), Gaussian blobs (each request carries its source), retire at estimated rel-L2 1e-6",
            "hbm_budget_bytes": budget,
            "batched_f32_ir": {k: summ[k] for k in keys}
                              | {k: summ[k] for k in ("ticks", "graph_captures", "graph_replays",
                                                      "graph_splits")
                                 if k in summ}
                              | {"true_rel_l2": err_stats(errs["batched"])},
            "batched_f32_ir_own_allocations": ({k: osum[k] for k in ("completed", "problems_per_s",
                                                                     "p50_latency_s", "makespan_s")}
                                               if osum else None),
            "one_at_a_time_f64": {k: bsum[k] for k in keys}
                                 | {"true_rel_l2": err_stats(errs["one_at_a_time"])},
            "speedup_problems_per_s": summ["problems_per_s"] / bsum["problems_per_s"],
            "at_0.8_capacity": {"arrival_rate_per_s": round(load, 3),
                                "batched_f32_ir": {k: lsum[k] for k in keys},
                                "one_at_a_time_f64": {k: lbase[k] for k in keys}}}


def say(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def extras_rates(lkp, torch, W, only: str = "") -> list:
    """Per-sweep rates of the other sets, orders, precisions and forms (with
    `only`: just the lines whose form contains that text)."""
    kn = 0.1
    cache = {}

    def src(kind, shape, seed):
        key = (kind, shape, seed)
        if key not in cache:
            cache.clear()
            cache[key] = W.poisson_source(kind, shape, seed=seed)
        return cache[key]

    s2 = lambda: src("blobs2d", (1024, 1024), 12345)
    s3 = lambda: src("blobs3d", (256, 256, 256), 12345)
    jobs = []   # (form, thunk)
    for N, lat in ORDERS.items():
        for prec in ("f64", "f32"):
            jobs.append(("population sweep", lambda N=N, lat=lat, prec=prec: dict(
                sweep_rate(lkp, torch, s2(), lat, N, prec, knudsen=kn, sweeps=200), grid="1024^2")))
    # generated minimal sets (square-symmetric shells) for the same orders
    for N, lat in ((5, "D2Q37"), (7, "D2Q77")):
        for prec in ("f64", "f32"):
            jobs.append(("generated set", lambda N=N, lat=lat, prec=prec: dict(
                sweep_rate(lkp, torch, s2(), lat, N, prec, knudsen=kn, sweeps=200),
                form="generated set", grid="1024^2")))
    # in place (one population buffer): every sweep pair gathers/scatters once
    for prec in ("f64", "f32"):
        jobs.append(("population sweep, in place", lambda prec=prec: dict(
            sweep_rate(lkp, torch, s2(), "D2Q81", 5, prec, knudsen=kn, sweeps=200, in_place=True),
            grid="1024^2")))
    for prec in ("f32", "f64"):
        jobs.append(("population sweep", lambda prec=prec: dict(
            sweep_rate(lkp, torch, s3(), "D3Q111", 5, prec, tau_lb=1.0, sweeps=40,
                       population_sweep=True), grid="256^3")))
        # the generated 3D set with 107 velocities, same problem
        jobs.append(("generated set", lambda prec=prec: dict(
            sweep_rate(lkp, torch, s3(), "D3Q107", 5, prec, tau_lb=1.0, sweeps=40,
                       population_sweep=True), grid="256^3", form="generated set")))
        jobs.append(("population sweep, in place", lambda prec=prec: dict(
            sweep_rate(lkp, torch, s3(), "D3Q111", 5, prec, tau_lb=1.0, sweeps=40,
                       population_sweep=True, in_place=True), grid="256^3")))

    # BF16 deviation storage (ablation): plain deviation sweeps; bytes = n_i
    # read + write (BF16), Phi read + write and S (FP32)
    def bf16dev():
        r = sweep_rate(lkp, torch, s2(), "D2Q81", 5, "bf16dev_ir", knudsen=kn, sweeps=200)
        bpc_dev = 4 * r_q(lkp, "D2Q81") + 12
        r.update(form="BF16 deviation storage", grid="1024^2",
                 gbs=s2().size * bpc_dev / (r["ms_per_sweep"] * 1e-3) / 1e9)
        r["frac_hbm"] = r["gbs"] / HBM_PEAK_GBS
        return r
    jobs.append(("BF16 deviation storage", bf16dev))
    # D3Q107 on the headline problem (512^3, Kn = 0.3, FP64, two buffers): the
    # same sweep with 4 fewer velocities (the headline line is D3Q111)
    jobs.append(("generated set", lambda: dict(
        sweep_rate(lkp, torch, src(C5["kind"], C5["shape"], C5["seed"]), "D3Q107", 5, "f64",
                   knudsen=C5["knudsen"], sweeps=20), grid="512^3", form="generated set")))

    # tau_lb = 1: the stencil form (state Phi, 3 values moved per cell)
    def stencil(prec):
        r = sweep_rate(lkp, torch, s3(), "D3Q111", 5, prec, tau_lb=1.0, sweeps=200)
        b = 4 if prec == "f32" else 8
        r.update(form="stencil (tau_lb=1)", grid="256^3",
                 gbs=s3().size * 3 * b / (r["ms_per_sweep"] * 1e-3) / 1e9)
        r["frac_hbm"] = r["gbs"] / HBM_PEAK_GBS
        return r
    for prec in ("f32", "f64"):
        jobs.append(("stencil (tau_lb=1)", lambda prec=prec: stencil(prec)))
    extras = [thunk() for form, thunk in jobs if only in form]
    return [{k: (round(v, 5) if isinstance(v, float) else v) for k, v in e.items()} for e in extras]


def extras_tts(lkp, torch, W) -> dict:
    """Time to solution, each answer checked against the oracle's fixed point."""
    out = {}
    # 64^2 standard LB (D2Q5, N = 1, tau_lb = 1), stop at max |dPhi| < 1e-10:
    # cache resident, reported as such
    s1 = W.poisson_source("sine", (64, 64))
    ref1 = oracle_fixed_point("D2Q5", 1, s1, tau_lb=1.0)
    with lkp.Problem(s1, "D2Q5", 1, tau_lb=1.0) as q:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rep = q.solve(tol_maxchange=1e-10, check_every=1, max_sweeps=100_000)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        phi = q.phi_host()
    out["c1_64x64_d2q5"] = {"rule": "max|dPhi| < 1e-10", "seconds": round(el, 4),
                            "sweeps": rep["sweeps"], "true_rel_l2": true_rel_l2(phi, ref1),
                            "phi_16_16": float(phi[16, 16]),
                            "note": "160 KB of populations: cache resident, launch bound"}
    # 256^3 D3Q111 N=5 at tau_lb = 1 (512 Gaussians + sine background): stencil
    # form, F32_IR and FP64, to rel-L2 1e-6 (the population sweep of the same
    # problem takes about two minutes: --configs)
    s3 = W.poisson_source("blobs3d", (256, 256, 256), seed=12345)
    ref3 = oracle_fixed_point("D3Q111", 5, s3, tau_lb=1.0)
    tts3 = []
    for prec in ("f32_ir", "f64"):
        tts3.append(dict(timed_solve(lkp, torch, s3, "D3Q111", 5, prec, 1e-6, ref=ref3, check_every=200,
                                     tau_lb=1.0), form="stencil (tau_lb=1)"))
    out["time_to_solution_256cubed"] = tts3
    del s3, ref3
    # 1024^2 D2Q81 N=5 Kn=0.1: FP64, FP32 + refinement, BF16 deviation + refinement
    s = W.poisson_source("blobs2d", (1024, 1024), seed=12345)
    ref = oracle_fixed_point("D2Q81", 5, s, knudsen=0.1)
    tts = []
    for prec, tol in (("f64", 1e-10), ("f32_ir", 1e-10), ("bf16dev_ir", 1e-10),
                      ("f64", 1e-6), ("f32_ir", 1e-6), ("bf16dev_ir", 1e-6)):
        tts.append(timed_solve(lkp, torch, s, "D2Q81", 5, prec, tol, ref=ref, knudsen=0.1))
    out["time_to_solution_1024x1024_d2q81"] = tts
    # advection-diffusion variant on the same grid: drift u = (0.05, 0.02)
    # (Peclet number |u| L / D ~ 0.6 at Kn = 0.1), rate and time to 1e-6
    from oracle import drift as DR
    from oracle import lattice as OL
    u = (0.05, 0.02)
    tau = OL.tau_from_knudsen(0.1, OL.get("D2Q81"), 1024)
    refd = DR.fixed_point("D2Q81", 5, tau, s, u)
    adv = []
    for prec in ("f64", "f32"):
        r = sweep_rate(lkp, torch, s, "D2Q81", 5, prec, knudsen=0.1, sweeps=200, drift=u)
        r.update(form="advection-diffusion", drift=u)
        adv.append({k: (round(v, 5) if isinstance(v, float) else v) for k, v in r.items()})
    for prec in ("f64", "f32_ir"):
        adv.append(dict(timed_solve(lkp, torch, s, "D2Q81", 5, prec, 1e-6, ref=refd, knudsen=0.1,
                                    drift=u), drift=u))
    out["advection_diffusion"] = adv
    return out


def configs_matrix(lkp, torch, W) -> dict:
    """The 1024^2 workload at every order and Knudsen number, FP64 and FP32 +
    refinement, to rel-L2 1e-6 with true errors; the 256^3 problem (tau_lb = 1)
    solved by population sweeps, FP32 + refinement and the BF16 deviation
    ablation as a separate run (each capped at 4 minutes of wall time)."""
    s = W.poisson_source("blobs2d", (1024, 1024), seed=12345)
    rows = []
    for N, lat in ORDERS.items():
        for kn in (0.01, 0.1, 0.5):
            ref = oracle_fixed_point(lat, N, s, knudsen=kn)
            for prec in ("f64", "f32_ir"):
                r = timed_solve(lkp, torch, s, lat, N, prec, 1e-6, ref=ref, knudsen=kn)
                r.update(lattice=lat, order=N, knudsen=kn)
                say(f"[configs] {lat} N={N} Kn={kn} {prec}: {r['seconds']} s, {r['sweeps']} sweeps, "
                    f"true {r['true_rel_l2']:.2e}")
                rows.append(r)
    s3 = W.poisson_source("blobs3d", (256, 256, 256), seed=12345)
    ref3 = oracle_fixed_point("D3Q111", 5, s3, tau_lb=1.0)
    abl = []
    for prec in ("bf16dev_ir", "f32_ir"):
        r = timed_solve(lkp, torch, s3, "D3Q111", 5, prec, 1e-6, ref=ref3, check_every=200,
                        chunk=2000, label="[configs] 256^3 population sweep", max_seconds=240.0,
                        tau_lb=1.0, population_sweep=True)
        say(f"[configs] 256^3 population sweep {prec}: {r['seconds']} s, true {r['true_rel_l2']:.2e}")
        abl.append(r)
    return {"c2_1024x1024": rows, "c3_256cubed_population_sweep": abl}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--chunk", type=int, default=50, help="sweeps per step")
    ap.add_argument("--no-extras", action="store_true", help="headline only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving stream")
    ap.add_argument("--serving-only", action="store_true",
                    help="headline and the serving stream only (no other extras)")
    ap.add_argument("--no-tts", action="store_true", help="skip the time-to-solution runs")
    ap.add_argument("--serve-requests", type=int, default=40)
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-sizes", choices=("scaled", "full"), default="scaled",
                    help="serving size mix: scaled (seconds) or full (up to 2048^2 and 256^3)")
    ap.add_argument("--c5-tts", action="store_true",
                    help="only the headline problem solved to --c5-tol: FP32+IR in place vs FP64 (long)")
    ap.add_argument("--c5-tol", type=float, default=1e-10)
    ap.add_argument("--c5-minutes", type=float, default=7.0, help="wall-time cap per solve")
    ap.add_argument("--configs", action="store_true",
                    help="only the order x Knudsen x precision matrix of the 1024^2 workload and "
                         "the 256^3 BF16 ablation (a few minutes)")
    ap.add_argument("--rates-only", action="store_true",
                    help="only the per-sweep rates of the other sets, precisions and forms "
                         "(counter runs of those kernels)")
    ap.add_argument("--skip-headline", action="store_true",
                    help="leave out the 512^3 headline (profiling the other parts only; the "
                         "printed line then carries no headline fields)")
    ap.add_argument("--only", default="",
                    help="with --rates-only: keep the rate lines whose form contains this text")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the sweep of "
              "a single problem runs on one device; sharding across GPUs is not implemented).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1504_05869_amd as lkp
    from paper_1504_05869_amd import workloads as W

    torch.cuda.set_device(0)
    if args.c5_tts:
        print(json.dumps({"stiff_512cubed": stiff_512(lkp, torch, args.c5_tol, 2000, args.c5_minutes)}),
              flush=True)
        return
    if args.configs:
        print(json.dumps({"configs": configs_matrix(lkp, torch, W)}), flush=True)
        return
    if args.calibrate_copy:
        x = torch.empty(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    if args.rates_only:
        print(json.dumps({"sweeps": extras_rates(lkp, torch, W, args.only)}), flush=True)
        return

    if args.skip_headline:
        out = {}
    else:
        out = headline(lkp, torch, args)
        say(f"headline: {out['value']} GLUPS, sweep {out['roofline']['achieved']} GB/s")
    if not args.no_extras and not args.serving_only:
        out["sweeps"] = extras_rates(lkp, torch, W)
        say("extras: rates done")
    if not args.no_extras and not args.serving_only and not args.no_tts:
        out.update(extras_tts(lkp, torch, W))
        say("extras: time to solution done")
    if (not args.no_extras or args.serving_only) and not args.no_serving:
        out["serving"] = serving_run(args.serve_requests, args.serve_rate,
                                     full_sizes=args.serve_sizes == "full")
        say("extras: serving done")
    if not args.no_cpu:
        # the oracle on the host cores, at the headline's set, order and
        # tau_lb, on 256^3 (512^3 in FP64 needs 238 GB of host memory)
        from oracle import lattice as OL
        tau = OL.tau_from_knudsen(C5["knudsen"], OL.get(C5["lattice"]), C5["shape"][0])
        s_cpu = W.poisson_source(C5["kind"], (256, 256, 256), seed=C5["seed"])
        out["cpu_baseline"] = cpu_baseline(s_cpu, C5["lattice"], C5["order"], tau, args.cpu_seconds,
                                           note=" (per-cell rate applies to the 512^3 workload)")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
