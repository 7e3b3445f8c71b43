"""Continuous-batching permeability server (host policy).

Requests (porous permeability solves of uneven sizes) arrive over time.  The
scheduler prepares each one on host threads (geometry), admits prepared
requests in arrival order while a slot is free and the device-memory budget
holds their footprint, runs all admitted lattices together K steps at a time
on the executor, and retires each lattice once its mean velocity is steady
(paper_1111_0922_amd.steady: converged, or at the rounding-noise floor of its
storage), once it diverges, or at `max_steps`.  Requests that arrive while
others run join at the next K-step boundary, so their work overlaps on the
device.

The loop keeps the device busy: while one run of K steps is in flight, the
scheduler admits the next requests, whose set-up (index build, equilibrium
start) the executor runs on a second stream; it then waits for the run,
retires finished lattices and starts the next run with the new ones in it.

The executor interface (GpuExecutor below; tests use a fake one):
    prepare(req)  -> footprint in bytes (host work, may run on a pool thread)
    admit(req)                          (allocates and initialises the lattice;
                                         it joins the batch at the next start)
    start(k)                            (k more steps of every admitted lattice, asynchronous)
    finish()      -> {rid: (M, Jx, Jy, Jz)} of the lattices in the run, after it
    release(req)                        (frees the lattice)
    busy_seconds  device time spent in runs so far
"""
from __future__ import annotations

import concurrent.futures as cf
import math
import time
from dataclasses import dataclass, field

import numpy as np

from .steady import CONVERGED, DIVERGED, NOISE_FLOOR, RUNNING, SteadyMonitor

CAP, OVERSIZE = "cap", "oversize"


@dataclass
class Request:
    rid: int
    seed: int
    arrival: float                      # seconds after the start of the run
    params: dict = field(default_factory=dict)
    footprint: int = 0
    n_fluid: int = 0
    n_cells: int = 0
    slot: int = -1
    admitted: float | None = None
    finished: float | None = None
    steps: int = 0
    velocity: float | None = None       # mass-weighted mean u_x at retirement
    permeability: float | None = None
    status: str = RUNNING               # converged, noise_floor, diverged, cap, oversize
    history: list = field(default_factory=list)

    @property
    def converged(self) -> bool:
        """Steady at retirement (converged or at its storage's noise floor)."""
        return self.status in (CONVERGED, NOISE_FLOOR)

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


def mean_velocity_x(mom, g):
    """U_x = (J_x + M g / 2) / M from FP64 moments (M, Jx, Jy, Jz)."""
    M = mom[0]
    return (mom[1] + 0.5 * M * g) / M


def poisson_arrivals(n, rate, seed):
    """n arrival times of a Poisson process of `rate` per second (exponential gaps, numpy PCG64)."""
    if not math.isfinite(rate) or rate <= 0:
        return np.zeros(n)
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, n)
    return np.cumsum(gaps) - gaps[0]


class Scheduler:
    def __init__(self, executor, *, hbm_budget: int, max_slots: int, k_steps: int = 100, tol: float = 1e-6,
                 max_steps: int = 20000, omega: float = 1.0, g: float = 1e-6, prep_threads: int = 4,
                 clock=None, sleep=None):
        if k_steps % 2:
            raise ValueError("k_steps must be even (the AA pattern's natural layout returns every 2 steps)")
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.k = int(k_steps)
        self.tol = float(tol)
        self.max_steps = int(max_steps)
        self.omega = float(omega)
        self.g = float(g)
        self.prep_threads = int(prep_threads)
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self.lups = 0             # lattice-node updates performed
        self.used = 0             # device bytes held by admitted requests
        self.peak_used = 0
        self.admission_order = []
        self.makespan = 0.0

    def _retire(self, r, status, u, now):
        r.status = status
        r.velocity = float(u)
        nu = (1.0 / self.omega - 0.5) / 3.0
        phi = r.n_fluid / r.n_cells if r.n_cells else float("nan")
        r.permeability = nu * phi * float(u) / self.g
        r.finished = now

    def serve(self, requests):
        """Serves `requests` (sorted by arrival); returns them with timings and results filled in."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending = list(reqs)
        preparing = {}
        ready = []
        active = {}               # rid -> request (admitted, not retired)
        monitors = {}
        in_flight = False
        t0 = self.clock()
        now = lambda: self.clock() - t0  # noqa: E731
        pool = cf.ThreadPoolExecutor(max_workers=self.prep_threads) if self.prep_threads > 0 else None
        try:
            while pending or preparing or ready or active:
                # arrivals -> preparation
                while pending and pending[0].arrival <= now():
                    r = pending.pop(0)
                    preparing[r.rid] = (r, pool.submit(self.ex.prepare, r) if pool else None)
                    if pool is None:
                        r.footprint = self.ex.prepare(r)
                for rid in list(preparing):
                    r, fut = preparing[rid]
                    if fut is None or fut.done():
                        if fut is not None:
                            r.footprint = int(fut.result())
                        del preparing[rid]
                        ready.append(r)
                ready.sort(key=lambda r: (r.arrival, r.rid))
                # admission (arrival order, slot and budget permitting), overlapping the run in flight
                while ready and len(active) < self.max_slots and self.used + ready[0].footprint <= self.budget:
                    r = ready.pop(0)
                    self.ex.admit(r)
                    r.admitted = now()
                    self.used += r.footprint
                    self.peak_used = max(self.peak_used, self.used)
                    active[r.rid] = r
                    monitors[r.rid] = SteadyMonitor(self.tol)
                    self.admission_order.append(r.rid)
                if ready and not active and ready[0].footprint > self.budget:
                    r = ready.pop(0)  # can never fit: fail it rather than stall the queue
                    r.finished = now()
                    r.status = OVERSIZE
                    continue
                if in_flight:
                    moms = self.ex.finish()
                    in_flight = False
                    for rid, m in moms.items():
                        r = active[rid]
                        r.steps += self.k
                        self.lups += r.n_fluid * self.k
                        u = mean_velocity_x(m, self.g)
                        r.history.append(float(u))
                        st = monitors[rid].push(u)
                        if st == RUNNING and r.steps >= self.max_steps:
                            st = CAP
                        if st != RUNNING:
                            self._retire(r, st, u, now())
                            self.ex.release(r)
                            self.used -= r.footprint
                            del active[rid], monitors[rid]
                if active:
                    self.ex.start(self.k)
                    in_flight = True
                elif not (pending or preparing or ready):
                    break
                else:
                    # idle: wait for the next arrival or preparation
                    nxt = pending[0].arrival - now() if pending else 0.001
                    self.sleep(max(min(nxt, 0.005), 0.0005))
        finally:
            if in_flight:
                self.ex.finish()
            if pool:
                pool.shutdown(wait=True)
        self.makespan = now()
        return reqs

    def report(self, reqs, warmup: int = 0, bytes_per_lup: float | None = None, hbm_peak_gbs: float = 8000.0):
        """Throughput and latency over the requests after the first `warmup` (by arrival).

        Latency percentiles are given over every finished request and, separately, over the steady
        ones (converged or at their noise floor); requests that hit the step cap, diverged or could
        never fit are counted, not hidden.
        """
        done = [r for r in reqs[warmup:] if r.finished is not None]
        steady = [r for r in done if r.converged]
        lat = np.array([r.latency for r in done]) if done else np.zeros(0)
        lat_s = np.array([r.latency for r in steady]) if steady else np.zeros(0)
        span = (max(r.finished for r in done) - min(r.arrival for r in done)) if done else 0.0
        busy = float(getattr(self.ex, "busy_seconds", float("nan")))
        pct = lambda a, q: float(np.percentile(a, q)) if len(a) else float("nan")  # noqa: E731
        out = {
            "requests": len(done),
            "converged": int(sum(r.status == CONVERGED for r in done)),
            "noise_floor": int(sum(r.status == NOISE_FLOOR for r in done)),
            "cap": int(sum(r.status == CAP for r in done)),
            "diverged": int(sum(r.status == DIVERGED for r in done)),
            "oversize": int(sum(r.status == OVERSIZE for r in done)),
            "solves_per_s": len(done) / span if span > 0 else float("nan"),
            "p50_latency_s": pct(lat, 50),
            "p99_latency_s": pct(lat, 99),
            "p50_latency_steady_s": pct(lat_s, 50),
            "p99_latency_steady_s": pct(lat_s, 99),
            "gpu_busy_frac": busy / self.makespan if self.makespan > 0 and math.isfinite(busy) else float("nan"),
            "mflups": self.lups / busy / 1e6 if busy > 0 else float("nan"),
            "peak_bytes": self.peak_used,
        }
        if bytes_per_lup and busy > 0:
            gbs = self.lups * bytes_per_lup / busy / 1e9
            out["GB/s"] = gbs
            out["frac_hbm"] = gbs / hbm_peak_gbs
            out["bytes_per_lup"] = bytes_per_lup
        return out


class GpuExecutor:
    """Executor on one GPU: each request a porous indirect AA lattice in one shared Batch.

    Runs go on the current stream; the set-up of admitted lattices (index build, binding,
    equilibrium start) goes on a second stream of default priority, so that it overlaps the run
    in flight.  The device time of every run is taken with events on the run's stream.
    """

    def __init__(self, max_slots=64, max_tiles=1 << 20, precision="f32", omega=1.0, g=1e-6, use_graph=True,
                 device=None):
        import torch

        from .batch import Batch
        self.torch = torch
        self.batch = Batch(max_slots, max_tiles, precision, use_graph=use_graph, device=device)
        self.device = self.batch.device
        self.setup_stream = torch.cuda.Stream(device=self.device)
        self.precision = precision
        self.omega = float(omega)
        self.g = float(g)
        self.grids = {}           # rid -> grid in the batch
        self.slots = {}           # rid -> slot
        self.joining = {}         # rid -> grid set up, joins at the next start
        self.masks = {}
        self.in_run = []          # rids of the run in flight
        self.events = None
        self.busy_seconds = 0.0
        self.pdf_size = {"f64": 8, "f32": 4, "f16s": 2, "f32s": 4}[precision]
        self.rank_lookup = False  # whether the admitted lattices look neighbour ids up by rank
        self.lattice_block = 0     # nodes per block of the admitted lattices (0: plain SoA)

    def prepare(self, req):
        import lbm_inputs
        mask, params = lbm_inputs.serving_geometry(req.seed)
        req.params = params
        req.n_cells = int(mask.size)
        req.n_fluid = int(mask.size - int(mask.sum(dtype=np.int64)))
        self.masks[req.rid] = mask
        nf = req.n_fluid + 1024   # the lattice covers whole blocks of 1024 nodes
        # lattice + IDX (with the slab order and the rank-lookup arrays: cell_of, 8 bytes per 32 cells) +
        # partials, and the cellmap held while the index is built
        return (19 * self.pdf_size + 19 * 4) * nf + 4 * req.n_cells + req.n_cells // 4 + 8192

    def admit(self, req):
        from .grid import Grid
        torch = self.torch
        e = req.params["edge"]
        with torch.cuda.stream(self.setup_stream):
            grid = Grid(e, e, e, addressing="indirect", precision=self.precision, omega=self.omega,
                        g=(self.g, 0.0, 0.0), f16_scale=1024.0, device=self.device)
            mask = torch.from_numpy(self.masks.pop(req.rid)).to(self.device, non_blocking=False)
            nf = grid.build_idx(mask)
            assert nf == req.n_fluid
            grid.cellmap = None   # the index is built; the cellmap is no longer needed
            grid._mask = None
            grid.bind("aa")
            grid.init_equilibrium()
            self.rank_lookup = grid.rank_lookup
            self.lattice_block = grid.lattice_block
        # the run stream reads this lattice only after the host has seen its set-up finish
        self.setup_stream.synchronize()
        self.joining[req.rid] = grid

    def start(self, k):
        torch = self.torch
        for rid, grid in self.joining.items():
            self.slots[rid] = self.batch.add(grid)
            self.grids[rid] = grid
        self.joining = {}
        self.in_run = list(self.grids)
        stream = torch.cuda.current_stream(self.device)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        self.batch.run_async(k)
        ev1.record(stream)
        self.events = (ev0, ev1)

    def finish(self):
        self.batch.last_status = self.batch.sync()
        ev0, ev1 = self.events
        self.busy_seconds += ev0.elapsed_time(ev1) * 1e-3
        m = self.batch.moments_host.numpy()
        return {rid: m[self.slots[rid]].copy() for rid in self.in_run}

    def release(self, req):
        slot = self.slots.pop(req.rid)
        self.batch.remove(slot)
        self.grids.pop(req.rid, None)
