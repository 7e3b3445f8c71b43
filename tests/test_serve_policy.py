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
    """Request r 'converges' after s_r steps: its mean velocity ramps linearly, then stays flat.
    A request whose seed is in `poison` returns non-finite moments (a diverged lattice)."""

    def __init__(self, clock, cost_per_step=1e-5, slots=8, poison=()):
        self.clock = clock
        self.cost = cost_per_step
        self.slots = slots
        self.poison = set(poison)
        self.active = {}
        self.joining = {}
        self.t = {}
        self.used = 0
        self.max_used = 0
        self.max_active = 0
        self.events = []
        self.busy_seconds = 0.0
        self.k = 0

    def prepare(self, req):
        req.n_fluid = 1000 * (1 + req.seed % 5)
        req.n_cells = 2 * req.n_fluid
        req.params = {"conv_steps": 200 + 100 * (req.seed % 7)}
        return 10 * req.n_fluid

    def admit(self, req):
        assert len(self.active) + len(self.joining) < self.slots
        self.joining[req.rid] = req
        self.t[req.rid] = 0
        self.used += req.footprint
        self.max_used = max(self.max_used, self.used)
        self.max_active = max(self.max_active, len(self.active) + len(self.joining))
        self.events.append(("admit", req.rid, self.clock()))

    def start(self, k):
        self.active.update(self.joining)
        self.joining = {}
        self.k = k

    def finish(self):
        dt = self.cost * self.k * len(self.active)
        self.clock.t += dt
        self.busy_seconds += dt
        out = {}
        for rid, req in self.active.items():
            self.t[rid] += self.k
            s = req.params["conv_steps"]
            U = 1e-3 * min(self.t[rid], s) / s
            out[rid] = np.array([1.0, U - 0.5 * G, 0.0, 0.0])
            if req.seed in self.poison and self.t[rid] >= 300:
                out[rid] = np.array([np.nan, np.nan, 0.0, 0.0])
        return out

    def release(self, req):
        del self.active[req.rid]
        self.used -= req.footprint
        self.events.append(("release", req.rid, self.clock()))


def _serve(n=40, rate=50.0, budget=60000, slots=8, poison=(), **kw):
    clock = FakeClock()
    ex = FakeExecutor(clock, slots=slots, poison=poison)
    sch = Scheduler(ex, hbm_budget=budget, max_slots=slots, k_steps=100, tol=1e-6, prep_threads=0, clock=clock,
                    sleep=clock.sleep, g=G, **kw)
    arr = poisson_arrivals(n, rate, seed=1)
    reqs = [Request(rid=i, seed=100 + i, arrival=float(a)) for i, a in enumerate(arr)]
    out = sch.serve(reqs)
    return sch, ex, out


def test_every_request_served_and_converged():
    sch, ex, out = _serve()
    assert all(r.finished is not None for r in out)
    assert all(r.converged and r.status == "converged" for r in out)
    for r in out:
        s = r.params["conv_steps"]
        # flat from the first K boundary at or after s steps; steady after three unchanged windows
        assert r.steps == (math.ceil(s / 100) + 3) * 100
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
    assert big.finished is not None and not big.converged and big.steps == 0 and big.status == "oversize"
    assert small.converged
    rep = sch.report(out)
    assert rep["oversize"] == 1 and rep["converged"] == 1


def test_max_steps_cap():
    sch, ex, out = _serve(n=5, max_steps=300)
    for r in out:
        assert r.steps <= 300
        if r.params["conv_steps"] >= 200:
            assert not r.converged and r.status == "cap"


def test_diverged_request_fails_alone():
    """A lattice whose moments turn non-finite is retired as diverged; every other request converges
    as it would without it."""
    _, _, ref = _serve(n=12, rate=100.0)
    sch, ex, out = _serve(n=12, rate=100.0, poison=(103, 107))
    by_rid = {r.rid: r for r in ref}
    for r in out:
        if r.seed in (103, 107):
            assert r.status == "diverged" and not r.converged and r.steps == 300
        else:
            assert r.status == "converged" and r.steps == by_rid[r.rid].steps
            assert r.velocity == by_rid[r.rid].velocity
    rep = sch.report(out)
    assert rep["diverged"] == 2 and rep["converged"] == 10
    assert ex.used == 0 and not ex.active


def test_report_percentiles():
    sch, ex, out = _serve()
    rep = sch.report(out)
    lat = np.array([r.latency for r in out])
    assert rep["requests"] == len(out)
    assert rep["p50_latency_s"] == pytest.approx(np.percentile(lat, 50))
    assert rep["p99_latency_s"] == pytest.approx(np.percentile(lat, 99))
    assert rep["p99_latency_s"] >= rep["p50_latency_s"] > 0
    assert rep["p50_latency_steady_s"] == pytest.approx(rep["p50_latency_s"])
    assert 0 < rep["gpu_busy_frac"] <= 1
    rep = sch.report(out, bytes_per_lup=188.0)
    assert rep["frac_hbm"] == pytest.approx(sch.lups * 188.0 / ex.busy_seconds / 1e9 / 8000.0)


def test_steady_monitor_tells_noise_from_approach():
    """A geometric approach with one overshoot converges (three small windows); a level with
    alternating rounding noise above tol is a noise floor; a NaN is a divergence."""
    from paper_1111_0922_amd.steady import SteadyMonitor
    m = SteadyMonitor(1e-7)
    u = [1.0 - 0.5 ** j * (1.0 if j < 6 else -0.3) for j in range(1, 60)]
    st = [m.push(x) for x in u]
    first = st.index("converged")
    assert "noise_floor" not in st[:first]
    assert all(abs(u[first - j] - u[first - j - 1]) < 1e-7 * u[first] for j in range(3))
    m = SteadyMonitor(1e-7)
    rng = np.random.default_rng(0)
    st = [m.push(1.0 + 5e-7 * rng.standard_normal()) for _ in range(40)]
    assert "noise_floor" in st and "converged" not in st[:st.index("noise_floor")]
    assert m.noise > 1e-7 and m.trend < 1e-7
    m = SteadyMonitor(1e-7)
    assert m.push(1.0) == "running" and m.push(float("nan")) == "diverged"


def test_mean_velocity_and_arrivals():
    assert mean_velocity_x(np.array([2.0, 1.0, 0, 0]), 0.5) == pytest.approx((1.0 + 0.5) / 2.0)
    a = poisson_arrivals(20000, 10.0, seed=3)
    assert a[0] == 0 and np.all(np.diff(a) >= 0)
    assert np.mean(np.diff(a)) == pytest.approx(0.1, rel=0.03)


def test_odd_k_rejected():
    with pytest.raises(ValueError):
        Scheduler(None, hbm_budget=1, max_slots=1, k_steps=99)
