"""Scheduler logic of the serving loop on the CPU, with a scripted backend.

The backend below stands in for the GPU: each admitted problem "converges"
after a number of ticks set by its size.  No solver arithmetic runs here; the
GPU path is covered by tests/test_gpu_serving.py.
"""
import math

import pytest

from paper_1504_05869_amd.serve import Request, Server, make_stream, summarize


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class ScriptedBackend:
    """Each tick costs `tick_cost` seconds of the fake clock; a problem needs
    ceil(cells / cells_per_tick) ticks."""

    def __init__(self, clock, tick_cost=0.01, cells_per_tick=40000):
        self.clock = clock
        self.tick_cost = tick_cost
        self.cells_per_tick = cells_per_tick
        self.resident = {}
        self.admitted_order = []
        self.cancelled = []
        self.max_resident_bytes = 0

    def footprint(self, req):
        return int(math.prod(req.shape)) * 100

    def admit(self, req, tol, max_sweeps):
        key = object()
        need = max(1, math.ceil(math.prod(req.shape) / self.cells_per_tick))
        self.resident[key] = [req, need, 0]
        self.admitted_order.append(req.rid)
        self.max_resident_bytes = max(self.max_resident_bytes,
                                      sum(self.footprint(r[0]) for r in self.resident.values()))
        return key

    def tick(self, sweeps):
        self.clock.t += self.tick_cost
        out = []
        for key, rec in list(self.resident.items()):
            rec[2] += 1
            state = "converged" if rec[2] >= rec[1] else "running"
            out.append((key, {"state": state, "status": "LKP_OK", "sweeps": rec[2] * sweeps,
                              "outer": 0, "est_rel_err": 1e-7}))
        return out

    def retire(self, key):
        del self.resident[key]
        return None

    def cancel(self, key):
        self.cancelled.append(self.resident[key][0].rid)
        del self.resident[key]


def _run(requests, budget, **kw):
    clock = FakeClock()
    be = ScriptedBackend(clock, **kw)
    srv = Server(be, budget, sweeps_per_tick=10, clock=clock, sleep=clock.sleep)
    res, summ = srv.run(requests)
    return be, srv, res, summ


def test_all_requests_retire_and_budget_is_respected():
    reqs = make_stream(60, rate=50.0, seed=1, sizes2d=((64, 64), (128, 128), (256, 256)),
                       sizes3d=((16, 16, 16), (32, 32, 32)))
    budget = 20_000_000
    be, srv, res, summ = _run(reqs, budget)
    assert summ["completed"] == 60
    assert be.max_resident_bytes <= budget
    assert srv.peak_used <= budget
    # FIFO admission
    assert be.admitted_order == sorted(be.admitted_order)
    for r in res:
        assert r.admitted >= r.arrival - 1e-12
        assert r.finished > r.admitted
    assert summ["p99_latency_s"] >= summ["p50_latency_s"] > 0


def test_problems_overlap_in_time():
    """Requests that arrive while others run are admitted before those finish."""
    reqs = [Request(i, 0.001 * i, (256, 256), "D2Q81", 5, 0.1, i, "blobs2d") for i in range(5)]
    be, srv, res, summ = _run(reqs, budget=10**12)
    assert max(r.admitted for r in res) < min(r.finished for r in res)
    # one tick advances all five: total ticks ~ ticks of one problem, not five
    assert srv.ticks <= 3 * math.ceil(256 * 256 / 40000)


def test_oversized_request_is_rejected_not_admitted():
    reqs = [Request(0, 0.0, (1024, 1024), "D2Q81", 5, 0.1, 0, "blobs2d"),
            Request(1, 0.0, (64, 64), "D2Q81", 5, 0.1, 1, "blobs2d")]
    be, srv, res, summ = _run(reqs, budget=1_000_000)
    assert res[0].status.startswith("rejected") and 0 not in be.admitted_order
    assert res[1].status == "converged"


def test_admission_waits_for_memory():
    reqs = [Request(i, 0.0, (128, 128), "D2Q81", 5, 0.1, i, "blobs2d") for i in range(4)]
    fp = 128 * 128 * 100
    be, srv, res, summ = _run(reqs, budget=2 * fp)
    assert srv.peak_used <= 2 * fp
    # the third request is admitted only after one of the first two retired
    first_done = min(res[0].finished, res[1].finished)
    assert res[2].admitted >= first_done


def test_idle_server_sleeps_until_next_arrival():
    reqs = [Request(0, 5.0, (64, 64), "D2Q81", 5, 0.1, 0, "blobs2d")]
    be, srv, res, summ = _run(reqs, budget=10**9)
    assert res[0].admitted >= 5.0 and res[0].finished > 5.0


def test_stream_is_seeded_and_poisson():
    a = make_stream(500, rate=10.0, seed=3)
    b = make_stream(500, rate=10.0, seed=3)
    assert [(r.arrival, r.shape, r.knudsen, r.seed) for r in a] == \
           [(r.arrival, r.shape, r.knudsen, r.seed) for r in b]
    gaps = [y.arrival - x.arrival for x, y in zip(a, a[1:])]
    assert abs(sum(gaps) / len(gaps) - 0.1) < 0.02
    assert all(0.05 <= r.knudsen <= 0.5 for r in a)


def test_summary_fields():
    from paper_1504_05869_amd.serve import Result
    rs = [Result(i, 0.0, 0.0, float(i + 1), status="converged") for i in range(100)]
    s = summarize(rs)
    assert s["completed"] == 100
    assert abs(s["p50_latency_s"] - 50.5) < 1e-9
    assert abs(s["p99_latency_s"] - 99.01) < 1e-9
    assert abs(s["problems_per_s"] - 1.0) < 1e-12


def test_deadline_expiry_cancels_and_frees():
    """A resident request past its deadline is cancelled after the tick that
    passes it and its memory goes to the next request; a queued request whose
    deadline passes while it waits for memory is cancelled unadmitted."""
    fp = 512 * 512 * 100
    reqs = [Request(0, 0.0, (512, 512), "D2Q81", 5, 0.1, 0, "blobs2d", deadline=0.015),
            Request(1, 0.0, (256, 256), "D2Q81", 5, 0.1, 1, "blobs2d", deadline=0.005),
            Request(2, 0.0, (64, 64), "D2Q81", 5, 0.1, 2, "blobs2d")]
    be, srv, res, summ = _run(reqs, budget=fp)
    # request 0 needs 7 ticks of 0.01 s: cancelled after the second, at t = 0.02
    assert res[0].status == "cancelled: deadline expired" and be.cancelled == [0]
    assert 0.015 <= res[0].finished <= 0.02 + 1e-12
    # request 1 waited for memory past its deadline: never admitted
    assert res[1].status.startswith("cancelled: deadline expired before admission")
    assert 1 not in be.admitted_order
    # request 2 took the freed memory and converged
    assert res[2].status == "converged" and res[2].admitted >= res[0].finished
    assert not be.resident and srv.peak_used <= fp
    assert summ["completed"] == 1
