"""Continuous-batching server for streams of Poisson problems.

Requests arrive over time (a seeded Poisson process).  The scheduler admits
them in arrival order while their device footprint fits the HBM budget, keeps
their populations resident, and advances all resident problems of a class
(lattice, order, precision) together, one batched group step per tick
(``lkp_group_step``: one launch per sweep covers many problems).  A problem
is retired as soon as its check says it reached the tolerance: its Phi is
read back, its memory freed, and newly arrived requests take the room.
Latency is arrival to retirement.

The scheduler talks to a backend object (``GpuBackend`` here); tests drive
the same scheduler with a scripted backend on the CPU.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the stream starts
    shape: tuple            # numpy order: (ny, nx) or (nz, ny, nx)
    lattice: str
    order: int
    knudsen: float
    seed: int
    kind: str               # workloads.poisson_source recipe
    deadline: float | None = None   # seconds after arrival; past it the request is cancelled
    source: np.ndarray | None = None  # the request's source field (else generated at admission)

    def source_field(self) -> np.ndarray:
        """The source this request carries, or the one its recipe and seed give."""
        if self.source is not None:
            return self.source
        from . import workloads as W
        return W.poisson_source(self.kind, self.shape, seed=self.seed)


def attach_sources(requests: list[Request]) -> list[Request]:
    """Generate every request's source field ahead of the stream, so that a
    request arrives carrying its data (the host work of synthesising inputs
    then stays out of the served timeline)."""
    for r in requests:
        if r.source is None:
            r.source = r.source_field()
    return requests


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    sweeps: int = 0
    outer: int = 0
    est_rel_err: float = float("nan")
    status: str = ""
    phi: np.ndarray | None = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def make_stream(n: int, rate: float, seed: int, sizes2d=((128, 128), (256, 256), (512, 512)),
                sizes3d=((32, 32, 32), (64, 64, 64)), kn=(0.05, 0.5),
                lattice2d="D2Q81", lattice3d="D3Q111", order=5) -> list[Request]:
    """Poisson arrivals at `rate` per second; sizes uniform over the 2D and 3D
    lists together; Kn ~ U(kn); Gaussian-blob sources (64 blobs of width 2 in
    2D, 512 of width 1.5 plus a sine background in 3D) with per-request seeds."""
    rng = np.random.default_rng(seed)
    sizes = [tuple(s) for s in sizes2d] + [tuple(s) for s in sizes3d]
    t = 0.0
    out = []
    for rid in range(n):
        t += rng.exponential(1.0 / rate)
        shape = sizes[rng.integers(len(sizes))]
        is3d = len(shape) == 3
        out.append(Request(rid, t, shape, lattice3d if is3d else lattice2d, order,
                           float(rng.uniform(*kn)), int(rng.integers(1 << 31)),
                           "blobs3d" if is3d else "blobs2d"))
    return out


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else float("nan")


class GpuBackend:
    """Resident problems on the GPU through the lkp library."""

    def __init__(self, precision: str = "f32_ir", keep_phi: bool = False, workspace: bool = True):
        """workspace: place each problem's state in a tensor from torch's
        caching allocator (admission and retirement then reuse cached device
        memory instead of allocating and freeing it each time)."""
        import paper_1504_05869_amd as lkp
        self.lkp = lkp
        self.precision = precision
        self.keep_phi = keep_phi
        self.workspace = bool(workspace)
        self.groups = {}

    def footprint(self, req: Request) -> int:
        return self.lkp.footprint_bytes(req.shape, req.lattice, req.order, knudsen=req.knudsen,
                                        precision=self.precision)

    def admit(self, req: Request, tol: float, max_sweeps: int):
        p = self.lkp.Problem(req.source_field(), req.lattice, req.order, knudsen=req.knudsen,
                             precision=self.precision, workspace=True if self.workspace else None)
        key = (req.lattice, req.order)
        g = self.groups.get(key)
        if g is None:
            g = self.groups[key] = self.lkp.Group(req.lattice, req.order, self.precision)
        g.add(p, tol_rel_l2=tol, max_sweeps=max_sweeps)
        return p

    def graph_stats(self) -> dict:
        """Captured graphs and graph-replayed steps over every group, and the
        velocity-group split each class's batched sweeps settled on."""
        tot = {"captures": 0, "replays": 0}
        for g in self.groups.values():
            for k, v in g.graph_stats().items():
                tot[k] += v
        tot["splits"] = {f"{lat} N={order}": g.split() for (lat, order), g in self.groups.items()}
        return tot

    def tick(self, sweeps: int):
        """One batched step of every non-empty group; (problem, report) pairs."""
        out = []
        for g in self.groups.values():
            if len(g):
                for r in g.step(sweeps):
                    out.append((r["problem"], r))
        return out

    def retire(self, p):
        phi = p.phi_host() if self.keep_phi else None
        self.cancel(p)
        return phi

    def cancel(self, p):
        """Take a problem out of its group and free its device state."""
        for g in self.groups.values():
            if p._h.value in g._members:
                g.remove(p)
        p.close()

    def close(self):
        for g in self.groups.values():
            g.close()
        self.groups.clear()


class Server:
    """Admission by footprint, batched ticks, retirement at tolerance;
    requests past their deadline are cancelled (queued ones before admission,
    resident ones after the tick that passes it) and their memory freed."""

    def __init__(self, backend, hbm_budget: int, sweeps_per_tick: int = 50, tol: float = 1e-6,
                 max_sweeps: int = 2_000_000, clock=time.perf_counter, sleep=time.sleep,
                 progress=None):
        self.progress = progress   # optional callable(str), called at each retirement
        self.backend = backend
        self.budget = int(hbm_budget)
        self.K = int(sweeps_per_tick)
        self.tol = float(tol)
        self.max_sweeps = int(max_sweeps)
        self.clock, self.sleep = clock, sleep
        self.peak_used = 0
        self.ticks = 0

    def run(self, requests: list[Request]) -> tuple[list[Result], dict]:
        reqs = sorted(requests, key=lambda r: r.arrival)
        results = {r.rid: Result(r.rid, r.arrival) for r in reqs}
        queue: list[Request] = []
        resident = {}            # problem -> (request, footprint)
        used = 0
        nxt = 0
        t0 = self.clock()
        cancel = getattr(self.backend, "cancel", self.backend.retire)

        def expired(req, t):
            return req.deadline is not None and t >= req.arrival + req.deadline

        while nxt < len(reqs) or queue or resident:
            now = self.clock() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                queue.append(reqs[nxt])
                nxt += 1
            for req in [q for q in queue if expired(q, now)]:
                queue.remove(req)
                results[req.rid].status = "cancelled: deadline expired before admission"
                results[req.rid].finished = now
            # FIFO admission while the footprint fits the budget
            while queue:
                req = queue[0]
                fp = self.backend.footprint(req)
                if fp > self.budget:
                    results[req.rid].status = "rejected: larger than the HBM budget"
                    results[req.rid].finished = self.clock() - t0
                    queue.pop(0)
                    continue
                if used + fp > self.budget:
                    break
                queue.pop(0)
                p = self.backend.admit(req, self.tol, self.max_sweeps)
                resident[p] = (req, fp)
                used += fp
                self.peak_used = max(self.peak_used, used)
                results[req.rid].admitted = self.clock() - t0
            if not resident:
                if nxt < len(reqs):
                    self.sleep(max(0.0, reqs[nxt].arrival - (self.clock() - t0)))
                continue
            self.ticks += 1
            for p, rep in self.backend.tick(self.K):
                if p not in resident:
                    continue
                if rep["state"] == "running":
                    req, fp = resident[p]
                    now = self.clock() - t0
                    if expired(req, now):
                        resident.pop(p)
                        cancel(p)
                        used -= fp
                        res = results[req.rid]
                        res.sweeps, res.outer = rep["sweeps"], rep["outer"]
                        res.est_rel_err = rep["est_rel_err"]
                        res.status = "cancelled: deadline expired"
                        res.finished = now
                    continue
                req, fp = resident.pop(p)
                res = results[req.rid]
                res.sweeps, res.outer = rep["sweeps"], rep["outer"]
                res.est_rel_err = rep["est_rel_err"]
                res.status = "converged" if rep["state"] == "converged" else rep["status"]
                res.phi = self.backend.retire(p)
                res.finished = self.clock() - t0
                used -= fp
                if self.progress:
                    self.progress(f"retired request {req.rid} {req.shape} {res.status} "
                                  f"sweeps {res.sweeps} at {res.finished:.2f} s")
        out = [results[r.rid] for r in reqs]
        extra = {"ticks": self.ticks, "peak_hbm_bytes": self.peak_used, "hbm_budget": self.budget}
        stats = getattr(self.backend, "graph_stats", None)
        if stats is not None:
            extra.update({"graph_" + k: v for k, v in stats().items()})
        return out, summarize(out, extra=extra)


def run_one_at_a_time(requests: list[Request], precision: str = "f64", tol: float = 1e-6,
                      check_every: int = 50, keep_phi: bool = False, clock=time.perf_counter,
                      sleep=time.sleep, progress=None) -> tuple[list[Result], dict]:
    """Baseline: the same trace solved one request at a time (lkp_solve)."""
    import paper_1504_05869_amd as lkp
    reqs = sorted(requests, key=lambda r: r.arrival)
    out = []
    t0 = clock()
    for req in reqs:
        now = clock() - t0
        if req.arrival > now:
            sleep(req.arrival - now)
        res = Result(req.rid, req.arrival, admitted=clock() - t0)
        with lkp.Problem(req.source_field(), req.lattice, req.order, knudsen=req.knudsen, precision=precision) as p:
            rep = p.solve(tol_rel_l2=tol, check_every=check_every, raise_on_error=False)
            res.sweeps, res.outer, res.est_rel_err = rep["sweeps"], rep["outer"], rep["est_rel_err"]
            res.status = "converged" if rep["status"] == 0 else str(rep["status"])
            if keep_phi:
                res.phi = p.phi_host()
        res.finished = clock() - t0
        out.append(res)
        if progress:
            progress(f"solved request {req.rid} {req.shape} {res.status} sweeps {res.sweeps} "
                     f"at {res.finished:.2f} s")
    return out, summarize(out)


def summarize(results: list[Result], extra: dict | None = None) -> dict:
    done = [r for r in results if r.status == "converged"]
    lat = [r.latency for r in done]
    span = (max(r.finished for r in done) - min(r.arrival for r in results)) if done else float("nan")
    d = {"requests": len(results), "completed": len(done),
         "problems_per_s": len(done) / span if done and span > 0 else float("nan"),
         "makespan_s": span, "p50_latency_s": percentile(lat, 50),
         "p99_latency_s": percentile(lat, 99), "mean_latency_s": float(np.mean(lat)) if lat else float("nan"),
         "sweeps_total": int(sum(r.sweeps for r in done))}
    if extra:
        d.update(extra)
    return d
