"""Benchmark of the lattice-kinetic Poisson sweep on one MI355X.

Workload (one GPU): periodic 1024 x 1024 grid, higher-order scheme at order
N = 5 on D2Q81, Kn = 0.1 (tau_lb = 118.26), FP64, source = 64 Gaussians of
width 2 cells with N(0,1) amplitudes at seeded uniform positions, mean removed.

A step is one pass of the solver's hot path: one chunk of --chunk sweeps
(fused pull-stream / moment / collide+source), the FP64 convergence
reductions on the last two sweeps, the read-back of the norms and the host's
stopping decision.  Inputs are resident in HBM before timing starts.

Printed: one JSON line with GLUPS (cell updates per second; one update moves
all Q populations of a cell), the roofline of the sweep kernel from HIP events
on the solver's stream, the oracle's CPU throughput on a bounded sample, and
extra measurements (other orders, FP32, 3D, time-to-solution).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
ORDERS = {1: "D2Q25", 3: "D2Q25", 5: "D2Q81", 7: "D2Q169"}


def bytes_per_cell(Q: int, precision: str) -> int:
    """Algorithmic HBM bytes of one sweep per cell (pull, two buffers):
    read Q populations + write Q populations + read S."""
    b = 8 if precision == "f64" else 4
    return 2 * b * Q + b


def r_q(lkp, lattice: str) -> int:
    return int(lkp.lattice_info(lattice)["Q"])


def sweep_rate(lkp, torch, s, lattice, order, precision, knudsen=None, tau_lb=None,
               sweeps=200, chunks=1, population_sweep=False, in_place=False, drift=None):
    """Average duration of one sweep (HIP events on the solver's stream)."""
    with lkp.Problem(s, lattice, order, knudsen=knudsen, tau_lb=tau_lb, precision=precision,
                     population_sweep=population_sweep, in_place=in_place, drift=drift) as p:
        p.step(2)
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


def cpu_baseline(s, lattice, order, tau, seconds=15.0):
    """Oracle C sweep (FP64, OpenMP) on the same grid for a bounded time."""
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
    return {"value": s.size * k / dt / 1e9, "unit": "GLUPS", "cores": SW.threads(),
            "kind": "oracle",
            "sample": f"{k} full sweeps of the {s.shape[1]}x{s.shape[0]} {lattice} N={order} "
                      f"FP64 grid in {dt:.1f} s"}


def stiff_512(lkp, torch, tol: float, chunk: int, minutes: float) -> dict:
    """512^3 D3Q111 N=5, Kn = 0.3 (tau_lb = 184.4), 4096 point-like Gaussians:
    FP32 sweeps + FP64 refinement (in place: 238 GB) against the plain FP64
    sweep (two buffers: 238 GB), each solved to estimated rel-L2 `tol`.  The
    solve runs as consecutive lkp_solve calls of `chunk` sweeps (a refinement
    stopped by max_sweeps keeps its partial correction and resumes from it),
    one progress line per call on stderr.  A solve still short of `tol` after
    `minutes` of wall time reports its reached error and the contraction rate,
    and a time extrapolated from that rate (labelled as such)."""
    from paper_1504_05869_amd import workloads as W
    shape = (512, 512, 512)
    t0 = time.perf_counter()
    s = W.poisson_source("stiff3d", shape, seed=5120)
    gen_s = time.perf_counter() - t0
    out = {"workload": "512^3 D3Q111 N=5 Kn=0.3, 4096 Gaussians sigma=1, amplitudes +-U(1,10), zero mean",
           "tol_rel_l2": tol, "source_generation_s": round(gen_s, 1), "runs": []}
    for prec, in_place in (("f32_ir", True), ("f64", False)):
        with lkp.Problem(s, "D3Q111", 5, knudsen=0.3, precision=prec, in_place=in_place) as q:
            info = q.info()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sweeps, outer, rep, hist = 0, 0, None, []
            while True:
                rep = q.solve(tol_rel_l2=tol, check_every=200, max_sweeps=chunk, raise_on_error=False)
                sweeps += rep["sweeps"]
                outer += rep["outer"]
                el = time.perf_counter() - t1
                hist.append((el, sweeps, rep["est_rel_err"]))
                print(f"[c5] {prec} in_place={in_place} {sweeps} sweeps {el:.0f} s est {rep['est_rel_err']:.3e} "
                      f"status {rep['status']}", file=sys.stderr, flush=True)
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
            out["runs"].append(run)
    return out


def serving_run(n_requests: int, rate: float, full_sizes: bool = False) -> dict:
    """Serving stream: continuous batching (FP32 + refinement) against the same
    trace solved one at a time in FP64, both to estimated rel-L2 1e-6.  The
    default size mix is scaled down so that the run takes seconds; full_sizes
    draws from {128..2048}^2 and {64,128,256}^3 with a 240 GiB HBM budget."""
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

    def say(msg):
        if full_sizes:
            print(f"[serving] {msg}", file=sys.stderr, flush=True)

    srv = serve.Server(serve.GpuBackend("f32_ir"), hbm_budget=budget, sweeps_per_tick=50,
                       tol=1e-6, progress=say)
    res, summ = srv.run(reqs)
    base, bsum = serve.run_one_at_a_time(reqs, "f64", tol=1e-6, check_every=50, progress=say)
    keys = ("completed", "problems_per_s", "p50_latency_s", "p99_latency_s", "makespan_s",
            "sweeps_total")
    sizes = ("{128,256,512,1024,2048}^2 and 3D D3Q111 N=5 {64,128,256}^3" if full_sizes else
             "{64,128,256,512}^2 and 3D D3Q111 N=5 {32,48,64}^3")
    return {"stream": f"{n_requests} requests, Poisson arrivals at {rate}/s, 2D D2Q81 N=5 "
                      f"{sizes}, Kn~U(0.05,0.5), Gaussian blobs, retire at estimated rel-L2 1e-6",
            "hbm_budget_bytes": budget,
            "batched_f32_ir": {k: summ[k] for k in keys}
                              | {k: summ[k] for k in ("ticks", "graph_captures", "graph_replays")
                                 if k in summ},
            "one_at_a_time_f64": {k: bsum[k] for k in keys},
            "speedup_problems_per_s": summ["problems_per_s"] / bsum["problems_per_s"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--chunk", type=int, default=100, help="sweeps per step")
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
    ap.add_argument("--c5", action="store_true",
                    help="only the 512^3 stiff workload: FP32+IR in place vs FP64 (long)")
    ap.add_argument("--c5-tol", type=float, default=1e-10)
    ap.add_argument("--c5-minutes", type=float, default=7.0, help="wall-time cap per solve")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build "
              "(the sweep of a single problem runs on one device).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1504_05869_amd as lkp
    from paper_1504_05869_amd import workloads as W

    torch.cuda.set_device(0)
    if args.c5:
        print(json.dumps({"stiff_512cubed": stiff_512(lkp, torch, args.c5_tol, 2000, args.c5_minutes)}),
              flush=True)
        return
    shape = (1024, 1024)
    lattice, order, kn, precision = "D2Q81", 5, 0.1, "f64"
    s = W.poisson_source("blobs2d", shape, seed=12345)
    n = s.size

    if args.calibrate_copy:
        x = torch.empty(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    p = lkp.Problem(s, lattice, order, knudsen=kn, precision=precision)
    info = p.info()
    Q = info["Q"]

    def step():
        # one chunk with the convergence check; the unreachable tolerance keeps
        # the solver going, so each call does exactly `chunk` sweeps
        return p.solve(tol_rel_l2=1e-300, max_sweeps=args.chunk, check_every=args.chunk,
                       use_graph=True, raise_on_error=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    last = None
    for _ in range(args.steps):
        last = step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sweeps = args.steps * args.chunk
    glups = n * sweeps / wall / 1e9
    # sweep kernel duration: events around plain sweeps on the same stream
    p.sync()
    k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    k0.record()
    p.step(args.chunk * 5)
    k1.record()
    k1.synchronize()
    ms_sweep = k0.elapsed_time(k1) / (args.chunk * 5)
    p.close()
    bpc = bytes_per_cell(Q, precision)
    achieved = n * bpc / (ms_sweep * 1e-3) / 1e9

    out = {
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
        "config": {"workload": "2D periodic 1024x1024 Poisson, D2Q81 N=5, Kn=0.1 "
                               f"(tau_lb={info['tau_lb']:.4f}), 64 Gaussians sigma=2, FP64",
                   "grid": [1024, 1024], "lattice": lattice, "order": order, "knudsen": kn,
                   "sweeps_per_step": args.chunk, "velocity_groups": info["velocity_groups"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("k_sweep_d2q81_f64_1024x1024"),
                     "kernel": "k_sweep (D2Q81, FP64)",
                     "bytes_per_launch": n * bpc, "ms_per_launch": round(ms_sweep, 5)},
        "paper_context": paper_context(),
        "last_check": {"est_rel_err": last["est_rel_err"], "rate": last["rate"]},
    }

    if not args.no_extras and not args.serving_only:
        extras = []
        for N, lat in ORDERS.items():
            for prec in ("f64", "f32"):
                r = sweep_rate(lkp, torch, s, lat, N, prec, knudsen=kn, sweeps=200)
                extras.append(r)
        # generated minimal sets (square-symmetric shells) for the same orders
        for N, lat in ((5, "D2Q37"), (7, "D2Q77")):
            for prec in ("f64", "f32"):
                extras.append(dict(sweep_rate(lkp, torch, s, lat, N, prec, knudsen=kn, sweeps=200),
                                   form="generated set"))
        # in place (one population buffer): every sweep pair gathers/scatters once
        for prec in ("f64", "f32"):
            extras.append(sweep_rate(lkp, torch, s, lattice, order, prec, knudsen=kn, sweeps=200,
                                     in_place=True))
        s3 = W.poisson_source("blobs3d", (256, 256, 256), seed=12345)
        for prec in ("f32", "f64"):
            extras.append(dict(sweep_rate(lkp, torch, s3, "D3Q111", 5, prec, tau_lb=1.0,
                                          sweeps=40, population_sweep=True), grid="256^3"))
            extras.append(dict(sweep_rate(lkp, torch, s3, "D3Q111", 5, prec, tau_lb=1.0,
                                          sweeps=40, population_sweep=True, in_place=True),
                               grid="256^3"))
        # BF16 deviation storage (ablation): plain deviation sweeps on the
        # headline problem; bytes = n_i read + write (BF16), Phi read + write
        # and S (FP32)
        r = sweep_rate(lkp, torch, s, lattice, order, "bf16dev_ir", knudsen=kn, sweeps=200)
        bpc_dev = 4 * r_q(lkp, lattice) + 12
        r.update(form="BF16 deviation storage", gbs=n * bpc_dev / (r["ms_per_sweep"] * 1e-3) / 1e9)
        r["frac_hbm"] = r["gbs"] / HBM_PEAK_GBS
        extras.append(r)
        # tau_lb = 1: the stencil form (state Phi, 3 values moved per cell)
        for prec in ("f32", "f64"):
            r = sweep_rate(lkp, torch, s3, "D3Q111", 5, prec, tau_lb=1.0, sweeps=200)
            b = 4 if prec == "f32" else 8
            r.update(form="stencil (tau_lb=1)", grid="256^3",
                     gbs=s3.size * 3 * b / (r["ms_per_sweep"] * 1e-3) / 1e9)
            r["frac_hbm"] = r["gbs"] / HBM_PEAK_GBS
            extras.append(r)
        out["sweeps"] = [{k: (round(v, 5) if isinstance(v, float) else v) for k, v in e.items()}
                         for e in extras]
    if not args.no_extras and not args.serving_only and not args.no_tts:
        # 256^3 D3Q111 N=5 at tau_lb = 1 (512 Gaussians + sine background):
        # time to rel-L2 1e-6 in FP32 + refinement and in FP64, stencil form
        s3 = W.poisson_source("blobs3d", (256, 256, 256), seed=12345)
        tts3 = []
        for prec in ("f32_ir", "f64"):
            with lkp.Problem(s3, "D3Q111", 5, tau_lb=1.0, precision=prec) as q:
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                rep = q.solve(tol_rel_l2=1e-6, check_every=200, max_sweeps=2_000_000)
                torch.cuda.synchronize()
                tts3.append({"precision": prec, "tol_rel_l2": 1e-6, "form": "stencil (tau_lb=1)",
                             "seconds": round(time.perf_counter() - t1, 4), "sweeps": rep["sweeps"],
                             "outer": rep["outer"], "est_rel_err": rep["est_rel_err"]})
        out["time_to_solution_256cubed"] = tts3
        del s3
    if not args.no_extras and not args.serving_only and not args.no_tts:
        # time-to-solution on the headline problem, FP64 and FP32 + refinement
        tts = []
        for prec, tol in (("f64", 1e-10), ("f32_ir", 1e-10), ("bf16dev_ir", 1e-10),
                          ("f64", 1e-6), ("f32_ir", 1e-6), ("bf16dev_ir", 1e-6)):
            with lkp.Problem(s, lattice, order, knudsen=kn, precision=prec) as q:
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                rep = q.solve(tol_rel_l2=tol, check_every=100, max_sweeps=2_000_000)
                torch.cuda.synchronize()
                tts.append({"precision": prec, "tol_rel_l2": tol,
                            "seconds": round(time.perf_counter() - t1, 4),
                            "sweeps": rep["sweeps"], "outer": rep["outer"],
                            "est_rel_err": rep["est_rel_err"]})
        out["time_to_solution"] = tts
        # advection-diffusion variant on the headline grid: drift u = (0.05, 0.02)
        # (Peclet number |u| L / D ~ 0.6 at Kn = 0.1), rate and time to 1e-6
        u = (0.05, 0.02)
        adv = []
        for prec in ("f64", "f32"):
            r = sweep_rate(lkp, torch, s, lattice, order, prec, knudsen=kn, sweeps=200, drift=u)
            r.update(form="advection-diffusion", drift=u)
            adv.append({k: (round(v, 5) if isinstance(v, float) else v) for k, v in r.items()})
        for prec in ("f64", "f32_ir"):
            with lkp.Problem(s, lattice, order, knudsen=kn, precision=prec, drift=u) as q:
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                rep = q.solve(tol_rel_l2=1e-6, check_every=100, max_sweeps=2_000_000)
                torch.cuda.synchronize()
                adv.append({"precision": prec, "tol_rel_l2": 1e-6, "drift": u,
                            "seconds": round(time.perf_counter() - t1, 4),
                            "sweeps": rep["sweeps"], "outer": rep["outer"],
                            "est_rel_err": rep["est_rel_err"]})
        out["advection_diffusion"] = adv

    if (not args.no_extras or args.serving_only) and not args.no_serving:
        out["serving"] = serving_run(args.serve_requests, args.serve_rate,
                                     full_sizes=args.serve_sizes == "full")

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(s, lattice, order, info["tau_lb"], args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
