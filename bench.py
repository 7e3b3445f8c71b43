#!/usr/bin/env python3
"""Benchmark: D3Q19 BGK node updates per second on one MI355X.

Headline (`value`): MFLUP/s of the AA pattern (SoA, direct addressing, FP64)
on the 256^3 channel (walls z = 0 and 255, periodic x and y, omega = 1.6,
body force 1e-6 in x, equilibrium start with +-1e-3 velocity noise).  A step
is one lattice time step (AA kernels alternate even/odd); the timed region
holds exactly --steps steps with the inputs resident in HBM.

Besides the headline the JSON line carries:
  roofline      achieved HBM bandwidth of the dominant kernel from its
                algorithmic bytes per launch and its event-timed average
                launch duration, against the 8 TB/s HBM3E peak;
  schemes       every scheme x layout on the same lattice, AA also in the library's default
                blocked order, in FP32, FP32-shifted and FP16-shifted storage, with the
                TRT collision, and on an indirect 256^3
                duct with a velocity inlet and a pressure outlet: whole-run MFLUP/s, and
                each kernel's event-timed duration, GB/s and fraction of the HBM peak
                (with its counted bytes while profiles/ is current for these kernels);
  porous512     every scheme on the 512^3 sphere pack (indirect addressing), the same way;
  copy          the STREAM-style copy bandwidth of the device;
  precision     the 384^3 sphere pack run to steady state in every storage form,
                with each form's permeability error against FP64;
  serving       continuous batching of porous solves: solves/s, p50/p99 latency,
                statuses, aggregate MFLUP/s and share of the HBM roofline (FP32 storage,
                and a saturated run in FP32-shifted storage beside it);
  cpu_baseline  the FP64 oracle timed on the host cores on bounded samples.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--only-main] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MFLUP/s D3Q19 AA (fp64/fp32, %HBM roofline); served solves/s + p99 latency"
# the kernels and their launch policy (block order, residency, kernel family: api.hip; batched
# launches: batch.hip): a change to any of them makes the committed counter summaries stale
KERNEL_SOURCES = ["kernels.hpp", "collide.hpp", "storage.hpp", "d3q19.hpp", "api.hip", "batch.hip"]


def kernel_hash() -> str:
    """Hash of the kernel sources' code: comments and blank space do not count,
    so a counter summary stays current until the code itself changes."""
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1111_0922_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)   # block comments
        text = re.sub(r"//[^\n]*", " ", text)                  # line comments
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def channel_grid(P, torch, n, scheme, layout, precision="f64", block=None):
    """The n^3 channel bound to `scheme`, velocity-noise start; `block` sets LBM_OPT_SOA_BLOCK."""
    import lbm_inputs
    grid = P.Grid(n, n, n, layout=layout, precision=precision, wall_z=True, omega=1.6, g=(1e-6, 0.0, 0.0),
                  f16_scale=1024.0)
    if block is not None:
        grid.set_option(P._lib.OPT_SOA_BLOCK, block)
    grid.bind(scheme)
    nf = grid.n_nodes
    u = torch.from_numpy(lbm_inputs.velocity_noise((n - 2, n, n), 1e-3, seed=1).reshape(3, -1))
    rho_u = torch.cat([torch.ones(1, nf, dtype=torch.float64), u], 0).cuda()
    grid.init_equilibrium(rho_u)
    del rho_u
    return grid


def time_steps(torch, grid, steps, warmup):
    grid.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grid.step(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def per_launch_ms(torch, grid, launches, collider="bgk"):
    """Average duration of single steps by parity, measured with events on the launch stream."""
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * launches)]
    per_kind = {0: [], 1: []}
    for k in range(launches):
        parity = grid.t & 1
        ev[2 * k].record(stream)
        grid.step(1, collider=collider)
        ev[2 * k + 1].record(stream)
        per_kind[parity].append(k)
    torch.cuda.synchronize()
    out = {}
    for parity, ks in per_kind.items():
        if ks:
            out[parity] = float(np.mean([ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in ks]))
    return out


# kernels one step launches, by step parity (the two-step scheme's collision and propagation
# kernels are timed together as one step)
STEP_KERNELS = {"ts": ("ts_step", "ts_step"), "os_push": ("os_push", "os_push"), "os_pull": ("os_pull", "os_pull"),
                "aa": ("aa_even", "aa_odd"), "et": ("et_even", "et_odd")}
PDF_SIZE = {"f64": 8, "f32": 4, "f16s": 2, "f32s": 4}
IDX_BYTES = {"ts_step": 72, "os_push": 72, "os_pull": 72, "aa_even": 0, "aa_odd": 72, "et_even": 28, "et_odd": 28}


def kernel_bytes(name, addressing, precision, nodes, rank=False, cells=0, et_rank=False):
    """Algorithmic HBM bytes of one launch (one step for ts_step): each PDF read and written once,
    no write-allocate, plus the IDX or esoteric-twist table entries an indirect kernel reads.  With
    neighbour ids looked up by rank, a kernel that reads them reads one 4-byte cell_of entry per node
    instead of 18 IDX entries, and the 8-byte words of ceil(cells / 32) once; the esoteric twist with
    its table from the words reads 4 bytes per node and the fluid and ghost words (16 bytes per 32
    cells) instead of its 28-byte table."""
    pdf = 2 * 19 * PDF_SIZE[precision] * (2 if name == "ts_step" else 1)
    if addressing != "indirect":
        return pdf * nodes
    if rank and IDX_BYTES[name] == 72:
        return (pdf + 4) * nodes + 8 * ((cells + 31) // 32)
    if et_rank and name.startswith("et"):   # the table from the rank words and the ghost words
        return (pdf + 4) * nodes + 16 * ((cells + 31) // 32)
    return (pdf + IDX_BYTES[name]) * nodes


def counter_table(workload):
    """{label: HBM bytes per launch} from profiles/counters_<workload>.md while its kernel hash is current."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.md")
    if not os.path.exists(path):
        return {}
    rows, current = {}, False
    with open(path) as fh:
        for line in fh:
            if line.startswith("kernel_source_hash:"):
                current = line.split(":", 1)[1].strip() == kernel_hash()
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) >= 8 and "/" in cells[0]:
                try:
                    rows[cells[0]] = float(cells[5])
                except ValueError:
                    pass
    return rows if current else {}


COPY_GBS = [None]   # the device's measured copy rate, once known (the paper's STREAM yardstick, Table 7)


def measure_row(P, torch, grid, scheme, addressing, precision, workload, steps=100, warmup=10, launches=40,
                collider="bgk", counters=None, layout="soa"):
    """Wall-clock MFLUP/s over `steps` steps, and every kernel's event-timed launch duration, achieved
    GB/s of its algorithmic bytes and fraction of the HBM peak (plus the counters' bytes if current)."""
    nodes = grid.n_nodes
    rank = addressing == "indirect" and grid.rank_lookup
    et_rank = addressing == "indirect" and grid.et_rank_lookup
    cells = int(np.prod(grid.shape))
    grid.step(warmup, collider=collider)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grid.step(steps, collider=collider)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    mf = nodes * steps / dt / 1e6
    bl = P.model_bytes(scheme, addressing, precision,
                       model="gpu_rank" if (et_rank if scheme == "et" else rank) else "gpu")
    blk = grid.lattice_block
    row = {"MFLUP/s": round(mf, 1), "bytes_per_lup": bl, "neighbour_ids": "rank" if rank else "idx",
           "storage": (f"soa in blocks of {blk}" if blk else layout), "GB/s": round(mf * bl / 1e3, 1),
           "frac_hbm_wall": round(mf * bl / 1e3 / HBM_PEAK_GBS, 4), "kernels": {}}
    ms = per_launch_ms(torch, grid, launches, collider)
    fr = []
    for parity, t in ms.items():
        name = STEP_KERNELS[scheme][parity]
        if name in row["kernels"]:
            continue
        t = float(np.mean([ms[p] for p in ms if STEP_KERNELS[scheme][p] == name]))
        b = kernel_bytes(name, addressing, precision, nodes, rank, cells, et_rank)
        k = {"ms": round(t, 4), "algorithmic_bytes": int(b), "GB/s": round(b / (t * 1e-3) / 1e9, 1),
             "frac_hbm": round(b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        if COPY_GBS[0]:
            k["frac_copy"] = round(b / (t * 1e-3) / 1e9 / COPY_GBS[0], 4)
        label = f"{workload}/{scheme}/{layout}/{precision}/{name}"
        if counters and label in counters:
            k["traffic"] = counters[label]
            k["traffic_over_algorithmic"] = round(counters[label] / b, 4)
        row["kernels"][name] = k
        fr.append(k["frac_hbm"])
    row["frac_hbm"] = min(fr)  # the slowest kernel's event-timed fraction
    return row


def pack_grid(P, torch, mask_t, scheme, n=512, precision="f64", omega=1.6):
    """The sphere pack on an indirect SoA grid bound to `scheme`, rest start."""
    g = P.Grid(n, n, n, addressing="indirect", precision=precision, omega=omega, g=(1e-6, 0, 0),
               et_ghosts=(scheme == "et"))
    g.build_idx(mask_t)
    g.cellmap = None
    g._mask = None
    g.bind(scheme)
    g.init_equilibrium()
    return g


CHANNEL_SET = [(sc, lay, "f64") for lay in ("soa", "aos") for sc in ("ts", "os_push", "os_pull", "aa", "et")] + \
              [("aa", "soa_blocked", "f64")] + [("aa", "soa", p) for p in ("f32", "f32s", "f16s")]
PACK_SET = [(sc, "soa", "f64") for sc in ("ts", "os_push", "os_pull", "aa", "et")]


def table_grid(P, torch, n, scheme, layout, prec):
    """The n^3 channel of one table row.  Row "soa" of the FP64 AA pattern runs plain SoA, as the
    headline does; row "soa_blocked" runs it in the library's default order for this lattice (4096-cell
    blocks); every other row runs the library's default order."""
    if layout == "soa_blocked":
        return channel_grid(P, torch, n, scheme, "soa", prec)
    plain = (scheme, layout, prec) == ("aa", "soa", "f64")
    return channel_grid(P, torch, n, scheme, layout, prec, block=0 if plain else None)


def profile_set(P, torch, which, steps, warmup, log):
    """Every kernel of one workload for a profiler: `warmup` + `steps` steps per configuration."""
    if which == "channel":
        for scheme, layout, prec in CHANNEL_SET:
            g = table_grid(P, torch, 256, scheme, layout, prec)
            dt = time_steps(torch, g, steps, warmup)
            print(json.dumps({"profile": f"channel256/{scheme}/{layout}/{prec}", "steps": steps,
                              "MFLUP/s": round(g.n_nodes * steps / dt / 1e6, 1)}), flush=True)
            del g
            torch.cuda.empty_cache()
    else:
        import lbm_inputs
        mask, _ = lbm_inputs.sphere_pack(512, 8, 0.40, seed=3)
        mask_t = torch.from_numpy(mask).cuda()
        del mask
        for scheme, layout, prec in PACK_SET:
            g = pack_grid(P, torch, mask_t, scheme)
            dt = time_steps(torch, g, steps, warmup)
            print(json.dumps({"profile": f"pack512/{scheme}/{layout}/{prec}", "steps": steps, "nodes": g.n_nodes,
                              "MFLUP/s": round(g.n_nodes * steps / dt / 1e6, 1)}), flush=True)
            del g
            torch.cuda.empty_cache()


def zband_column_order(grid, n, band=8):
    """Block-order table for lbm_set_block_order on an n^3 lexicographic indirect grid: z-bands of
    `band` planes, band k on XCD k mod 8, each XCD sweeping its bands column by column (y, then the
    band's z), so that the rows z +- 1 of a block run right after it."""
    import torch
    cm = grid.cellmap[: n ** 3].cpu().numpy()
    cells = np.flatnonzero(cm >= 0)
    T = (len(cells) + 255) // 256
    first = cells[::256][:T]
    y0, z0 = (first // n) % n, first // (n * n)
    tiles = np.arange(T)
    xcd = (z0 // band) % 8
    lists = [tiles[xcd == x][np.lexsort((tiles[xcd == x], z0[xcd == x], y0[xcd == x], (z0 // band)[xcd == x]))]
             for x in range(8)]
    m = min(len(lst) for lst in lists)
    order = np.empty(T, np.int64)
    for x in range(8):
        order[x: 8 * m: 8] = lists[x][:m]
    rest = np.sort(np.concatenate([lst[m:] for lst in lists]))
    order[8 * m:] = rest
    return torch.from_numpy(order.astype(np.int32)).cuda()


PACK_ORDERS = [("lexicographic, natural order", None, 0, False), ("lexicographic, XCD slab order", None, -1, False),
               ("lexicographic, z-band columns", None, 0, True), ("bands nx x 16 x nz, XCD slab order", (512, 16, 512), -1, False)]


def profile_orders(P, torch, log, launches=4):
    """AA FP64 on the 512^3 pack under the block orders and numberings of PACK_ORDERS, in that
    sequence: `launches` even and odd steps each (for a counter pass), then event-timed launches."""
    import lbm_inputs
    mask, _ = lbm_inputs.sphere_pack(512, 8, 0.40, seed=3)
    mask_t = torch.from_numpy(mask).cuda()
    del mask
    for name, brick, slab, columns in PACK_ORDERS:
        g = P.Grid(512, 512, 512, addressing="indirect", omega=1.6, g=(1e-6, 0, 0), brick=brick)
        g.build_idx(mask_t)
        g.set_option(P._lib.OPT_SLAB_ORDER, slab)
        if columns:
            g.set_block_order(zband_column_order(g, 512))
        g.cellmap = None
        g._mask = None
        g.bind("aa")
        g.init_equilibrium()
        g.step(2 * launches)
        ms = per_launch_ms(torch, g, 20)
        print(json.dumps({"profile_order": name, "aa_even_ms": round(ms[0], 4), "aa_odd_ms": round(ms[1], 4)}),
              flush=True)
        del g
        torch.cuda.empty_cache()


def bench_copy(P, torch, nbytes=4 << 30, reps=10):
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    P.stream_copy(src, dst)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        P.stream_copy(src, dst)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del src, dst
    return 2 * nbytes / dt / 1e9


def cpu_info():
    """Host CPU model, sockets and cores from lscpu (empty values if it is missing)."""
    import subprocess
    info = {}
    try:
        text = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        text = ""
    for line in text.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            info[k.strip()] = v.strip()
    return {"model": info.get("Model name", ""), "sockets": info.get("Socket(s)", ""),
            "cores_per_socket": info.get("Core(s) per socket", ""), "threads_per_core": info.get("Thread(s) per core", ""),
            "cpus": info.get("CPU(s)", str(os.cpu_count()))}


def cpu_baseline():
    """The FP64 oracle (two-step two-grid, dense lattice) timed on the host, one thread and all threads.

    Samples (bounded, ~20 s of CPU work):
      config1  32^3 channel, omega 1, 100 steps in full;
      config2  256^3 channel, omega 1.6: 2 steps on all threads; one thread: 1 step of a
               256 x 256 x 34 channel (32 fluid planes, the same per-node work);
      config3  the first 32 z-planes of the 512^3 sphere pack (r 8, porosity 0.40, seed 3), periodic:
               2 steps on all threads, 1 step on one;
      config4  the first 32 z-planes of the 384^3 sphere pack (r 8, porosity 0.6, seed 4): 2 / 1 steps.
    A step's time is that of a call with the steps less that of a call with none (the oracle copies
    its lattice in and allocates the second one on every call).  `value` is config2 on all threads.
    """
    import lbm_inputs
    import oracle
    oracle.build(force=False)
    all_threads = oracle.num_threads(0)
    g = (1e-6, 0.0, 0.0)

    def rate(f, solid, omega, steps, threads):
        t0 = time.perf_counter()
        oracle.run_ts(f, solid, 0, omega, g, threads=threads)
        t_over = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.run_ts(f, solid, steps, omega, g, threads=threads)
        dt = max(time.perf_counter() - t0 - t_over, 1e-9)
        nf = int((solid == 0).sum())
        return {"MFLUP/s": round(nf * steps / dt / 1e6, 2), "steps": steps, "threads": threads, "seconds": round(dt, 2)}

    out = {}
    solid = lbm_inputs.channel_mask(32, 32, 32)
    f = oracle.init_equilibrium(lbm_inputs.rho_u_field(solid.shape,
                                                       lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=1)), solid)
    out["config1_32cube_channel"] = {"all": rate(f, solid, 1.0, 100, all_threads), "one": rate(f, solid, 1.0, 100, 1)}
    solid = lbm_inputs.channel_mask(256, 256, 256)
    f = oracle.init_equilibrium(lbm_inputs.rho_u_field(solid.shape), solid)
    c2 = {"all": rate(f, solid, 1.6, 2, all_threads)}
    solid = lbm_inputs.channel_mask(256, 256, 34)
    f = oracle.init_equilibrium(lbm_inputs.rho_u_field(solid.shape), solid)
    c2["one"] = rate(f, solid, 1.6, 1, 1)
    c2["one"]["sample"] = "256 x 256 x 34 channel"
    out["config2_256cube_channel"] = c2
    del f
    for key, (n, phi, seed, omega) in (("config3_512pack_32planes", (512, 0.40, 3, 1.6)),
                                        ("config4_384pack_32planes", (384, 0.6, 4, 1.0))):
        solid = np.ascontiguousarray(lbm_inputs.sphere_pack(n, 8, phi, seed)[0][:32])
        f = oracle.init_equilibrium(lbm_inputs.rho_u_field(solid.shape), solid)
        out[key] = {"all": rate(f, solid, omega, 2, all_threads), "one": rate(f, solid, omega, 1, 1)}
        del f
    head = out["config2_256cube_channel"]["all"]
    return {"value": head["MFLUP/s"], "unit": "MFLUP/s", "cores": all_threads, "kind": "oracle",
            "sample": f"256^3 channel, FP64 two-step (pull), {head['steps']} steps on {all_threads} threads "
                      "(config1 in full; configs 2-4 sampled, one thread and all threads)",
            "configs": out, "cpu": cpu_info()}


def serving_bench(log, n_requests, n_light=100, n_shifted=300, seed_base=100000):
    """Porous permeability solves of uneven sizes (FP32 AA indirect), continuous batching.

    Three runs: all `n_requests` at t = 0 (saturated), then Poisson arrivals at 0.9x and 0.5x of the
    saturated rate (`n_requests` and `n_light` requests).  The first tenth of each run's requests,
    by arrival, is warm-up and left out of the figures.  A fourth run serves the first `n_shifted`
    of the same requests saturated in FP32 words holding the deviation f - w (F32S: the same bytes
    per update, far less rounding), whose flows reach the steady state in fewer steps.
    """
    import paper_1111_0922_amd as P
    from paper_1111_0922_amd.serve import GpuExecutor, Request, Scheduler, poisson_arrivals
    def run(rate, seed0, n, precision="f32"):
        ex = GpuExecutor(max_slots=64, max_tiles=1 << 20, precision=precision, omega=1.0, g=1e-6)
        sch = Scheduler(ex, hbm_budget=64 << 30, max_slots=64, k_steps=100, tol=1e-6, max_steps=20000,
                        omega=1.0, g=1e-6, prep_threads=8)
        arr = poisson_arrivals(n, rate, seed=seed0)
        reqs = [Request(rid=i, seed=seed0 + i, arrival=float(a)) for i, a in enumerate(arr)]
        out = sch.serve(reqs)
        # the bytes the batched kernels move: IDX or the neighbour-id lookup by rank, as the slots ran
        bl = P.model_bytes("aa", "indirect", precision, model="gpu_rank" if ex.rank_lookup else "gpu")
        rep = sch.report(out, warmup=n // 10, bytes_per_lup=bl, hbm_peak_gbs=HBM_PEAK_GBS)
        rep["neighbour_ids"] = "rank" if ex.rank_lookup else "idx"
        rep["rate_per_s"] = rate
        rep["arrived"] = n
        rep["warmup_discarded"] = n // 10
        rep["steps_mean"] = float(np.mean([r.steps for r in out]))
        rep["makespan_s"] = sch.makespan
        rep["storage"] = precision
        rep["lattice_block"] = ex.lattice_block
        rep["permeability"] = {r.seed: r.permeability for r in out}
        log(f"[bench]   {rep['requests']} measured requests, {rep['solves_per_s']:.2f} solves/s, "
            f"p50 {rep['p50_latency_s']:.2f} s, p99 {rep['p99_latency_s']:.2f} s, "
            f"{rep['mflups']:.0f} MFLUP/s, busy {rep['gpu_busy_frac']:.3f}")
        return rep

    log(f"[bench] serving: saturated ({n_requests} requests at t=0)")
    sat = run(float("inf"), seed_base, n_requests)
    out = {"saturated": sat}
    for frac, n in ((0.9, n_requests), (0.5, n_light)):
        lam = frac * sat["solves_per_s"]
        log(f"[bench] serving: Poisson rate {lam:.2f}/s ({frac} x saturated), {n} requests")
        out[f"poisson_{frac}"] = run(lam, seed_base + 1000 * int(frac * 10), n)
    if n_shifted > 0:
        log(f"[bench] serving: saturated, FP32 shifted storage ({n_shifted} requests at t=0)")
        out["saturated_f32s"] = run(float("inf"), seed_base, n_shifted, "f32s")
        # the same requests' permeabilities in the two storages
        k32, k32s = out["saturated"]["permeability"], out["saturated_f32s"]["permeability"]
        d = np.array([abs(k32[s_] - k32s[s_]) / abs(k32s[s_]) for s_ in k32s if s_ in k32])
        out["saturated_f32s"]["permeability_rel_diff_vs_f32"] = {"median": float(np.median(d)), "max": float(d.max())}
    for run_ in out.values():
        if isinstance(run_, dict):
            run_.pop("permeability", None)
    out["budget_bytes"] = 64 << 30
    out["max_slots"] = 64
    out["storage"] = "f32"
    out["bytes_per_lup"] = out["saturated"]["bytes_per_lup"]
    return out


PERMEABILITY_BOUNDS = {"f32": 1e-2, "f32s": 1e-5, "f16s_sigma1": 5e-3, "f16s_sigma1024": 1e-4}


def precision_study(log, n=384, radius=8, porosity=0.6, seed=4, tol=1e-7, max_steps=20000, k=100):
    """384^3 sphere pack (r 8, porosity 0.6), AA indirect to steady state in every storage form.

    Steady state: the mean velocity U, sampled every k steps, changes by less than tol of itself over
    three consecutive windows (converged), or has no trend above tol per window while its window
    changes keep flipping sign (noise floor: steady to the storage's rounding noise), or the cap.
    Reported per form: steps, status, permeability and its relative error against FP64 with the
    stated bound, mass drift, MFLUP/s and the fraction of the HBM roofline (model bytes per LUP).
    """
    import torch
    import lbm_inputs
    import paper_1111_0922_amd as P
    from paper_1111_0922_amd.steady import SteadyMonitor
    mask, spheres = lbm_inputs.sphere_pack(n, radius, porosity, seed)
    mt = torch.from_numpy(mask).cuda()
    phi = float(1 - mask.mean())
    del mask
    g, omega = 1e-6, 1.0
    nu = (1.0 / omega - 0.5) / 3.0
    res = {"lattice": f"{n}^3", "radius": radius, "porosity": phi, "spheres": spheres, "omega": omega, "g": g,
           "tol": tol, "window_steps": k, "max_steps": max_steps,
           "rule": "converged: 3 consecutive windows with |dU|/U < tol; noise_floor: least-squares trend "
                   "< tol per window over 10 windows with >= 3 sign flips of dU; else cap"}
    for prec, sigma in (("f64", 1.0), ("f32", 1.0), ("f32s", 1.0), ("f16s", 1.0), ("f16s", 1024.0)):
        key = prec if prec != "f16s" else f"f16s_sigma{int(sigma)}"
        grid = P.Grid(n, n, n, addressing="indirect", precision=prec, omega=omega, g=(g, 0, 0), f16_scale=sigma)
        nf = grid.build_idx(mt)
        grid.bind("aa")
        grid.init_equilibrium()
        m0 = grid.moments().cpu().numpy()
        mon, steps = SteadyMonitor(tol), 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while steps < max_steps and mon.status == "running":
            grid.step(k)
            steps += k
            m = grid.moments().cpu().numpy()
            mon.push((m[1] + 0.5 * m[0] * g) / m[0])
        dt = time.perf_counter() - t0
        U = mon.history[-1]
        mf = nf * steps / dt / 1e6
        bl = P.model_bytes("aa", "indirect", prec, model="gpu_rank" if grid.rank_lookup else "gpu")
        res[key] = {"steps": steps, "status": mon.status if mon.status != "running" else "cap",
                    "U": U, "permeability": nu * phi * U / g, "MFLUP/s": round(mf, 1),
                    "frac_hbm": round(mf * bl / 1e3 / HBM_PEAK_GBS, 4), "bytes_per_lup": bl,
                    "neighbour_ids": "rank" if grid.rank_lookup else "idx", "lattice_block": grid.lattice_block,
                    "mass_drift": float(abs(m[0] - m0[0]) / m0[0]),
                    "last_window_change": mon.last_change, "trend_per_window": mon.trend,
                    "noise_per_window": mon.noise}
        log(f"[precision] {key}: {steps} steps, {res[key]['status']}, k = {res[key]['permeability']:.8g}, "
            f"{mf:.0f} MFLUP/s")
        del grid
        torch.cuda.empty_cache()
    k64 = res["f64"]["permeability"]
    for key, bound in PERMEABILITY_BOUNDS.items():
        e = abs(res[key]["permeability"] - k64) / abs(k64)
        res[key]["rel_err_vs_f64"] = e
        res[key]["bound"] = bound
        res[key]["within_bound"] = bool(e <= bound)
    res["nodes"] = nf
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--only-main", action="store_true", help="headline AA run only (for profiling)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--serving-requests", type=int, default=500,
                    help="requests of the saturated and 0.9x Poisson serving runs (0 = skip serving)")
    ap.add_argument("--serving-light", type=int, default=100, help="requests of the 0.5x Poisson serving run")
    ap.add_argument("--precision-study", action="store_true",
                    help="only the 384^3 steady-state precision study (FP64 / FP32 / FP16-shifted)")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision study")
    ap.add_argument("--profile-aa", choices=["f64", "f32", "f32s", "f16s"], default=None,
                    help="only the AA 256^3 channel run in this storage (for profiling)")
    ap.add_argument("--profile-porous", action="store_true",
                    help="only AA FP64 on the 512^3 sphere pack, indirect addressing (for profiling)")
    ap.add_argument("--profile-set", choices=["channel", "pack"], default=None,
                    help="only every kernel of the 256^3 channel (10 scheme x layout, AA FP32/F32S/FP16S) or of "
                         "the 512^3 pack (5 schemes), --warmup + --steps steps each (for profiling)")
    ap.add_argument("--profile-orders", action="store_true",
                    help="only AA FP64 on the 512^3 pack under several block orders and numberings (profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the copy kernel on 1 GiB, 3 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(sharding over GPUs is a design, not built)", file=sys.stderr)
        sys.exit(2)
    if args.steps % 2:
        args.steps += 1  # whole even/odd pairs

    import torch
    import paper_1111_0922_amd as P

    if args.calibrate_copy:
        nbytes = 1 << 30
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            P.stream_copy(src, dst)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "lbm_stream_copy", "bytes_read": nbytes, "bytes_written": nbytes,
                          "launches": 3}), flush=True)
        return

    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    if args.profile_aa:
        grid = channel_grid(P, torch, 256, "aa", "soa", args.profile_aa, block=0)
        dt = time_steps(torch, grid, args.steps, args.warmup)
        print(json.dumps({"profile": f"AA SoA {args.profile_aa} 256^3 channel", "steps": args.steps,
                          "MFLUP/s": round(grid.n_nodes * args.steps / dt / 1e6, 1)}), flush=True)
        return
    if args.profile_porous:
        import lbm_inputs
        mask, _ = lbm_inputs.sphere_pack(512, 8, 0.40, seed=3)
        grid = P.Grid(512, 512, 512, addressing="indirect", omega=1.6, g=(1e-6, 0, 0))
        nf = grid.build_idx(torch.from_numpy(mask).cuda())
        del mask
        grid.bind("aa")
        grid.init_equilibrium()
        dt = time_steps(torch, grid, args.steps, args.warmup)
        print(json.dumps({"profile": "AA SoA f64 indirect 512^3 sphere pack", "nodes": nf, "steps": args.steps,
                          "MFLUP/s": round(nf * args.steps / dt / 1e6, 1)}), flush=True)
        return
    if args.precision_study:
        print(json.dumps({"precision_study": precision_study(log)}), flush=True)
        return
    if args.profile_set:
        profile_set(P, torch, args.profile_set, args.steps, args.warmup, log)
        return
    if args.profile_orders:
        profile_orders(P, torch, log)
        return

    n = 256
    log(f"[bench] AA SoA FP64 256^3 channel: warmup {args.warmup}, steps {args.steps}")
    grid = table_grid(P, torch, n, "aa", "soa", "f64")   # plain SoA, the layout the paper measures
    nf = grid.n_nodes
    m0 = grid.moments().cpu().numpy()
    dt = time_steps(torch, grid, args.steps, args.warmup)
    ms_per_step = dt / args.steps * 1e3
    mflups = nf * args.steps / dt / 1e6
    m1 = grid.moments().cpu().numpy()
    b_lup = P.model_bytes("aa", "direct", "f64")
    launch = per_launch_ms(torch, grid, 200)
    dom = max(launch, key=lambda k: launch[k])
    kname = "aa_even" if dom == 0 else "aa_odd"
    bytes_per_launch = b_lup * nf
    achieved = bytes_per_launch / (launch[dom] * 1e-3) / 1e9
    traffic = counter_table("channel256").get(f"channel256/aa/soa/f64/{kname}")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname,
                "avg_launch_ms": {("aa_even" if k == 0 else "aa_odd"): round(v, 4) for k, v in launch.items()},
                "algorithmic_bytes_per_launch": int(bytes_per_launch),
                "algorithmic_bytes_per_lup": b_lup}
    del grid
    torch.cuda.empty_cache()

    result = {"metric": METRIC, "value": round(mflups, 1), "unit": "MFLUP/s", "n_gpus": 1,
              "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
              "data": "synthetic",
              "config": {"workload": "D3Q19 BGK 256^3 channel (walls z=0,255; periodic x,y), direct addressing, "
                                     "SoA, AA pattern, omega 1.6, g 1e-6 x",
                         "nodes": nf, "lattice": "256x256x256", "layout": "soa", "storage": "plain soa",
                         "addressing": "direct", "scheme": "aa"},
              "roofline": roofline,
              "mass_drift": float(abs(m1[0] - m0[0]) / m0[0]),
              # the paper's measured numbers: CPU nodes, FP64 TRT, indirect SoA (Sec. 10); context only
              "paper_context": {"aa_MLUP_s": ">100", "hardware": "2-socket Westmere (2x Xeon X5650, 12 cores)",
                                "workload": "FP64 TRT, indirect addressing, SoA, channel and packed bed",
                                "source": "Sec. 10 (text; the figures' curves are not available)"}}

    if not args.only_main:
        log("[bench] copy calibration")
        result["copy"] = {"GB/s": round(bench_copy(P, torch), 1)}
        COPY_GBS[0] = result["copy"]["GB/s"]
        roofline["frac_of_copy"] = round(roofline["achieved"] / COPY_GBS[0], 4)
        log("[bench] scheme x layout table, 256^3 channel (FP64; AA also FP32, F32S, FP16S)")
        table = {}
        cc = counter_table("channel256")
        for scheme, layout, prec in CHANNEL_SET:
            g = table_grid(P, torch, n, scheme, layout, prec)
            key = f"{scheme}/{layout}" + ("" if prec == "f64" else f"/{prec}")
            table[key] = measure_row(P, torch, g, scheme, "direct", prec, "channel256", counters=cc, layout=layout,
                                     steps=100 if prec == "f64" else 200)
            del g
            torch.cuda.empty_cache()
            log(f"[bench]   {key}: {table[key]['MFLUP/s']:.0f} MFLUP/s, slowest kernel {table[key]['frac_hbm']:.3f} of HBM")
        # the paper's collision (TRT, Lambda = 3/16) on the headline's kernels
        g = channel_grid(P, torch, n, "aa", "soa", block=0)
        table["aa/soa/trt"] = measure_row(P, torch, g, "aa", "direct", "f64", "channel256", collider="trt", steps=200)
        del g
        torch.cuda.empty_cache()
        log(f"[bench]   aa/soa/trt: {table['aa/soa/trt']['MFLUP/s']:.0f} MFLUP/s")
        # open boundaries: 256^3 duct (indirect), velocity inlet x = 0, pressure outlet x = 255,
        # walls z = 0 and z = 255, periodic in y
        duct = np.zeros((n, n, n), np.uint8)
        duct[:, :, 0] = 2
        duct[:, :, n - 1] = 3
        duct[0] = 1
        duct[n - 1] = 1
        g = P.Grid(n, n, n, addressing="indirect", omega=1.6)
        g.build_idx(torch.from_numpy(duct).cuda())
        g.set_boundary(1, "velocity", 1.0, (0.01, 0.0, 0.0))
        g.set_boundary(2, "pressure", 1.0, (0.01, 0.0, 0.0))
        g.bind("aa")
        g.init_equilibrium()
        key = "aa/indirect/duct_open_boundaries"
        table[key] = measure_row(P, torch, g, "aa", "indirect", "f64", "duct256", steps=200)
        del g, duct
        torch.cuda.empty_cache()
        log(f"[bench]   {key}: {table[key]['MFLUP/s']:.0f} MFLUP/s")
        result["schemes"] = table

        log("[bench] 512^3 sphere pack (r 8, porosity 0.40), indirect, FP64, every scheme")
        import lbm_inputs
        mask, spheres = lbm_inputs.sphere_pack(512, 8, 0.40, seed=3)
        porous = {"spheres": spheres, "porosity": float(1 - mask.mean())}
        mask_t = torch.from_numpy(mask).cuda()
        del mask
        cp = counter_table("pack512")
        for scheme, layout, prec in PACK_SET:
            g = pack_grid(P, torch, mask_t, scheme)
            porous["nodes"] = g.n_nodes
            porous[scheme] = measure_row(P, torch, g, scheme, "indirect", prec, "pack512", counters=cp)
            del g
            torch.cuda.empty_cache()
            log(f"[bench]   {scheme}: {porous[scheme]['MFLUP/s']:.0f} MFLUP/s, "
                f"slowest kernel {porous[scheme]['frac_hbm']:.3f} of HBM")
        result["porous512"] = porous
        del mask_t
        torch.cuda.empty_cache()
        if not args.no_precision:
            log("[bench] precision study: 384^3 sphere pack to steady state, every storage form")
            result["precision"] = precision_study(log)
        if args.serving_requests > 0:
            result["serving"] = serving_bench(log, args.serving_requests, args.serving_light)

    if not args.no_cpu and not args.only_main:
        log("[bench] CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline()

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
