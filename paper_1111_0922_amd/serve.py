"""Continuous-batching permeability server (host policy).

Requests (porous permeability solves of uneven sizes) arrive over time.  The
scheduler prepares each one on host threads (geometry), admits prepared
requests in arrival order while a slot is free and the device-memory budget
holds their footprint, runs all admitted lattices together K steps at a time
on the executor, and retires each lattice once its mean velocity has
converged (relative change per K steps below `tol`) or `max_steps` is
reached.  Requests that arrive while others run join at the next K-step
boundary, so their work overlaps on the device.

The executor interface (GpuExecutor below; tests use a fake one):
    prepare(req)  -> footprint in bytes (host work, may run on a pool thread)
    admit(req)    -> slot               (allocates and initialises the lattice)
    run(k)        -> {slot: (M, Jx, Jy, Jz)} after k more steps of every slot
    release(req)                        (frees the lattice)
"""
from __future__ import annotations

import concurrent.futures as cf
import math
import time
from dataclasses import dataclass, field

import numpy as np


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
    converged: bool = False
    history: list = field(default_factory=list)

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
        self.busy = 0.0           # time spent inside executor.run
        self.lups = 0             # lattice-node updates performed
        self.used = 0             # device bytes held by admitted requests
        self.peak_used = 0
        self.admission_order = []

    def _converged(self, req):
        h = req.history
        if req.steps >= self.max_steps:
            return True, False
        if len(h) >= 2 and h[-1] != 0.0 and math.isfinite(h[-1]):
            if abs(h[-1] - h[-2]) / abs(h[-1]) < self.tol:
                return True, True
        if not math.isfinite(h[-1]):
            return True, False
        return False, False

    def serve(self, requests):
        """Serves `requests` (sorted by arrival); returns them with timings and results filled in."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending = list(reqs)
        preparing = {}
        ready = []
        active = {}
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
                # admission: arrival order, slot and budget permitting
                while ready and len(active) < self.max_slots and self.used + ready[0].footprint <= self.budget:
                    r = ready.pop(0)
                    r.slot = self.ex.admit(r)
                    r.admitted = now()
                    self.used += r.footprint
                    self.peak_used = max(self.peak_used, self.used)
                    active[r.slot] = r
                    self.admission_order.append(r.rid)
                if ready and not active and ready[0].footprint > self.budget:
                    r = ready.pop(0)  # can never fit: fail it rather than stall the queue
                    r.finished = now()
                    r.converged = False
                    continue
                if active:
                    t_run = self.clock()
                    moms = self.ex.run(self.k)
                    self.busy += self.clock() - t_run
                    for slot, r in list(active.items()):
                        r.steps += self.k
                        self.lups += r.n_fluid * self.k
                        u = mean_velocity_x(moms[slot], self.g)
                        r.history.append(float(u))
                        done, conv = self._converged(r)
                        if done:
                            r.velocity = float(u)
                            nu = (1.0 / self.omega - 0.5) / 3.0
                            phi = r.n_fluid / r.n_cells if r.n_cells else float("nan")
                            r.permeability = nu * phi * float(u) / self.g
                            r.converged = conv
                            r.finished = now()
                            self.ex.release(r)
                            self.used -= r.footprint
                            del active[slot]
                else:
                    # idle: wait for the next arrival or preparation
                    nxt = pending[0].arrival - now() if pending else 0.001
                    self.sleep(max(min(nxt, 0.005), 0.0005))
        finally:
            if pool:
                pool.shutdown(wait=True)
        self.makespan = now()
        return reqs

    def report(self, reqs, warmup: int = 0):
        done = [r for r in reqs[warmup:] if r.finished is not None]
        lat = np.array([r.latency for r in done]) if done else np.zeros(0)
        span = (max(r.finished for r in done) - min(r.arrival for r in done)) if done else 0.0
        return {
            "requests": len(done),
            "converged": int(sum(r.converged for r in done)),
            "solves_per_s": len(done) / span if span > 0 else float("nan"),
            "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else float("nan"),
            "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else float("nan"),
            "gpu_busy_frac": self.busy / self.makespan if getattr(self, "makespan", 0) else float("nan"),
            "mflups": self.lups / self.busy / 1e6 if self.busy > 0 else float("nan"),
            "peak_bytes": self.peak_used,
        }


class GpuExecutor:
    """Executor on one GPU: each request a porous indirect AA lattice in one shared Batch."""

    def __init__(self, max_slots=64, max_tiles=1 << 20, precision="f32", omega=1.0, g=1e-6, use_graph=True,
                 device=None):
        import torch

        from .batch import Batch
        self.torch = torch
        self.batch = Batch(max_slots, max_tiles, precision, use_graph=use_graph, device=device)
        self.precision = precision
        self.omega = float(omega)
        self.g = float(g)
        self.grids = {}
        self.masks = {}
        self.pdf_size = {"f64": 8, "f32": 4, "f16s": 2, "f32s": 4}[precision]

    def prepare(self, req):
        import lbm_inputs
        mask, params = lbm_inputs.serving_geometry(req.seed)
        req.params = params
        req.n_cells = int(mask.size)
        req.n_fluid = int(mask.size - int(mask.sum(dtype=np.int64)))
        self.masks[req.rid] = mask
        nf = req.n_fluid + 128
        # lattice + IDX + partials, and the cellmap held while the index is built
        return (19 * self.pdf_size + 18 * 4) * nf + 4 * req.n_cells + 4096

    def admit(self, req):
        from .grid import Grid
        torch = self.torch
        e = req.params["edge"]
        grid = Grid(e, e, e, addressing="indirect", precision=self.precision, omega=self.omega,
                    g=(self.g, 0.0, 0.0), f16_scale=1024.0)
        mask = torch.from_numpy(self.masks.pop(req.rid)).to(self.batch.device)
        nf = grid.build_idx(mask)
        assert nf == req.n_fluid
        grid.cellmap = None   # the index is built; the cellmap is no longer needed
        grid._mask = None
        grid.bind("aa")
        grid.init_equilibrium()
        slot = self.batch.add(grid)
        self.grids[slot] = grid
        return slot

    def run(self, k):
        m = self.batch.run(k)
        return {s: m[s] for s in self.grids}

    def release(self, req):
        self.batch.remove(req.slot)
        self.grids.pop(req.slot, None)
