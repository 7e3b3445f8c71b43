"""Serving policy on the CPU: a fake executor and a fake clock stand in for the GPU."""
import math

import numpy as np
import pytest

from paper_1111_0922_amd.serve import Request, Scheduler, mean_velocity_x, poisson_arrivals

G = 1e-6


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-4)


class FakeExecutor:
    """Request r 'converges' after s_r steps: its mean velocity ramps linearly, then stays flat."""

    def __init__(self, clock, cost_per_step=1e-5, slots=8):
        self.clock = clock
        self.cost = cost_per_step
        self.free = list(range(slots))
        self.active = {}
        self.t = {}
        self.used = 0
        self.max_used = 0
        self.max_active = 0
        self.events = []

    def prepare(self, req):
        req.n_fluid = 1000 * (1 + req.seed % 5)
        req.n_cells = 2 * req.n_fluid
        req.params = {"conv_steps": 200 + 100 * (req.seed % 7)}
        return 10 * req.n_fluid

    def admit(self, req):
        slot = self.free.pop(0)
        self.active[slot] = req
        self.t[slot] = 0
        self.used += req.footprint
        self.max_used = max(self.max_used, self.used)
        self.max_active = max(self.max_active, len(self.active))
        self.events.append(("admit", req.rid, self.clock()))
        return slot

    def run(self, k):
        self.clock.t += self.cost * k * len(self.active)
        out = {}
        for slot, req in self.active.items():
            self.t[slot] += k
            s = req.params["conv_steps"]
            U = 1e-3 * min(self.t[slot], s) / s
            out[slot] = np.array([1.0, U - 0.5 * G, 0.0, 0.0])
        return out

    def release(self, req):
        del self.active[req.slot]
        self.free.append(req.slot)
        self.free.sort()
        self.used -= req.footprint
        self.events.append(("release", req.rid, self.clock()))


def _serve(n=40, rate=50.0, budget=60000, slots=8, **kw):
    clock = FakeClock()
    ex = FakeExecutor(clock, slots=slots)
    sch = Scheduler(ex, hbm_budget=budget, max_slots=slots, k_steps=100, tol=1e-6, prep_threads=0, clock=clock,
                    sleep=clock.sleep, g=G, **kw)
    arr = poisson_arrivals(n, rate, seed=1)
    reqs = [Request(rid=i, seed=100 + i, arrival=float(a)) for i, a in enumerate(arr)]
    out = sch.serve(reqs)
    return sch, ex, out


def test_every_request_served_and_converged():
    sch, ex, out = _serve()
    assert all(r.finished is not None for r in out)
    assert all(r.converged for r in out)
    for r in out:
        s = r.params["conv_steps"]
        # flat after s steps; detected at the first K boundary with two equal readings
        assert r.steps == (math.ceil(s / 100) + 1) * 100
        assert abs(r.velocity - 1e-3) < 1e-15


def test_budget_and_slots_never_exceeded():
    sch, ex, _ = _serve(budget=45000, slots=4)
    assert ex.max_used <= 45000
    assert ex.max_active <= 4
    assert sch.peak_used <= 45000


def test_admission_in_arrival_order():
    sch, ex, out = _serve()
    by_arrival = [r.rid for r in sorted(out, key=lambda r: (r.arrival, r.rid))]
    assert sch.admission_order == by_arrival


def test_continuous_batching_overlaps_requests():
    """A request that arrives while others run joins before they finish."""
    sch, ex, out = _serve(n=20, rate=200.0)
    admits = {rid: t for kind, rid, t in ex.events if kind == "admit"}
    releases = {rid: t for kind, rid, t in ex.events if kind == "release"}
    overlapped = sum(1 for a in out for b in out if a.rid < b.rid and admits[b.rid] < releases[a.rid])
    assert overlapped > 0
    assert ex.max_active > 1


def test_oversized_request_fails_without_blocking():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    sch = Scheduler(ex, hbm_budget=25000, max_slots=8, prep_threads=0, clock=clock, sleep=clock.sleep, g=G)
    reqs = [Request(rid=0, seed=104, arrival=0.0), Request(rid=1, seed=100, arrival=0.0)]  # 50000 B, 10000 B
    out = sch.serve(reqs)
    big = [r for r in out if r.rid == 0][0]
    small = [r for r in out if r.rid == 1][0]
    assert big.finished is not None and not big.converged and big.steps == 0
    assert small.converged


def test_max_steps_cap():
    sch, ex, out = _serve(n=5, max_steps=300)
    for r in out:
        assert r.steps <= 300
        if r.params["conv_steps"] >= 300:
            assert not r.converged


def test_report_percentiles():
    sch, ex, out = _serve()
    rep = sch.report(out)
    lat = np.array([r.latency for r in out])
    assert rep["requests"] == len(out)
    assert rep["p50_latency_s"] == pytest.approx(np.percentile(lat, 50))
    assert rep["p99_latency_s"] == pytest.approx(np.percentile(lat, 99))
    assert rep["p99_latency_s"] >= rep["p50_latency_s"] > 0
    assert 0 < rep["gpu_busy_frac"] <= 1


def test_mean_velocity_and_arrivals():
    assert mean_velocity_x(np.array([2.0, 1.0, 0, 0]), 0.5) == pytest.approx((1.0 + 0.5) / 2.0)
    a = poisson_arrivals(20000, 10.0, seed=3)
    assert a[0] == 0 and np.all(np.diff(a) >= 0)
    assert np.mean(np.diff(a)) == pytest.approx(0.1, rel=0.03)


def test_odd_k_rejected():
    with pytest.raises(ValueError):
        Scheduler(None, hbm_budget=1, max_slots=1, k_steps=99)
