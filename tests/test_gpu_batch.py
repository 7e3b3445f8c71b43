"""Batched AA executor: each lattice evolves to the same bits alone and in any mix."""
import numpy as np
import pytest
import torch

import lbm_inputs
import oracle
from lbm_cases import from_device, rel_err, to_device

pytestmark = pytest.mark.gpu

GEOMS = [((20, 20, 20), 3, 0.55, 11), ((28, 24, 31), 4, 0.45, 12), ((36, 36, 36), 5, 0.7, 13),
         ((17, 9, 13), 2, 0.6, 14)]


def _grid(shape, r, phi, seed, precision, omega=1.0, g=1e-5):
    import paper_1111_0922_amd as P
    solid = lbm_inputs.sphere_pack(shape, r, phi, seed)[0]
    nz, ny, nx = solid.shape
    grid = P.Grid(nx, ny, nz, addressing="indirect", precision=precision, omega=omega, g=(g, 0, 0))
    grid.build_idx(torch.from_numpy(solid).cuda())
    grid.bind("aa")
    rho_u = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=seed))
    grid.init_equilibrium(to_device(rho_u.reshape(4, -1)[:, solid.reshape(-1) == 0]))
    return grid, solid


@pytest.mark.parametrize("precision", ["f32", "f64", "f16s", "f32s"])
@pytest.mark.parametrize("use_graph", [True, False])
def test_alone_equals_mixed_bitwise(precision, use_graph):
    import paper_1111_0922_amd as P
    K = 20
    # alone: lbm_step + lbm_reduce_moments, one lattice at a time (one starts at odd parity)
    alone = []
    for i, gm in enumerate(GEOMS):
        grid, _ = _grid(*gm, precision)
        if i == 1:
            grid.step(1)
        for _ in range(2):
            grid.step(K)
        alone.append((from_device(grid.get_pdfs()), from_device(grid.moments())))
        del grid
    # mixed: all in one batch, two runs of K steps
    batch = P.Batch(8, 4096, precision, use_graph=use_graph)
    grids = []
    for i, gm in enumerate(GEOMS):
        grid, _ = _grid(*gm, precision)
        if i == 1:
            grid.step(1)
        grids.append((batch.add(grid), grid))
    for _ in range(2):
        m = batch.run(K)
    for (slot, grid), (f_alone, m_alone) in zip(grids, alone):
        assert np.array_equal(from_device(grid.get_pdfs()).view(np.int64), f_alone.view(np.int64)), slot
        assert np.array_equal(m[slot].view(np.int64), m_alone.view(np.int64)), slot


def test_slot_churn_stays_exact():
    import paper_1111_0922_amd as P
    K = 10
    batch = P.Batch(4, 2048, "f32", use_graph=True)
    g0, _ = _grid(*GEOMS[0], "f32")
    g1, _ = _grid(*GEOMS[1], "f32")
    s0, s1 = batch.add(g0), batch.add(g1)
    batch.run(K)
    batch.remove(s1)                      # g1 leaves after K steps
    g2, _ = _grid(*GEOMS[2], "f32")
    s2 = batch.add(g2)                    # g2 joins at t = 0 while g0 is at t = K
    assert s2 == s1                       # freed slot is reused
    m = batch.run(K)
    assert g0.t == 2 * K and g1.t == K and g2.t == K
    # reference evolutions, one lattice each
    for grid, gm, steps in ((g0, GEOMS[0], 2 * K), (g1, GEOMS[1], K), (g2, GEOMS[2], K)):
        ref, _ = _grid(*gm, "f32")
        ref.step(steps)
        assert np.array_equal(from_device(grid.get_pdfs()).view(np.int64), from_device(ref.get_pdfs()).view(np.int64))
    ref2, _ = _grid(*GEOMS[2], "f32")
    ref2.step(K)
    assert np.array_equal(m[s2], from_device(ref2.moments()))


def test_batch_fp64_matches_oracle():
    import paper_1111_0922_amd as P
    (shape, r, phi, seed) = GEOMS[3]
    grid, solid = _grid(shape, r, phi, seed, "f64", omega=1.6)
    f0 = from_device(grid.get_pdfs())
    batch = P.Batch(2, 64, "f64", use_graph=True)
    slot = batch.add(grid)
    m = batch.run(12)
    dense = np.zeros((19,) + solid.shape)
    dense.reshape(19, -1)[:, solid.reshape(-1) == 0] = f0
    want = oracle.run_ts(dense, solid, 12, 1.6, (1e-5, 0, 0))
    assert rel_err(from_device(grid.get_pdfs()), oracle.fluid_view(want, solid)) <= 1e-12
    mo = oracle.moments(want, solid)
    assert abs(m[slot][0] - mo[0]) / mo[0] <= 1e-13


def test_batch_rejects_unsupported_grids():
    import paper_1111_0922_amd as P
    batch = P.Batch(2, 64, "f32")
    direct = P.Grid(8, 8, 8, precision="f32", wall_z=True)
    direct.bind("aa")
    with pytest.raises(P.LbmError):
        batch.add(direct)
    g64, _ = _grid(*GEOMS[0], "f64")
    with pytest.raises(P.LbmError):
        batch.add(g64)


def test_serving_end_to_end_small():
    """A few real requests through the scheduler and the GPU executor (steps capped)."""
    from paper_1111_0922_amd.serve import GpuExecutor, Request, Scheduler
    ex = GpuExecutor(max_slots=4, max_tiles=1 << 16, precision="f32")
    sch = Scheduler(ex, hbm_budget=8 << 30, max_slots=4, k_steps=100, tol=1e-6, max_steps=600, prep_threads=2)
    reqs = [Request(rid=i, seed=7000 + i, arrival=0.02 * i) for i in range(5)]
    out = sch.serve(reqs)
    rep = sch.report(out)
    assert rep["requests"] == 5
    for r in out:
        assert r.steps > 0 and r.finished is not None
        assert np.isfinite(r.permeability) and r.permeability > 0
    assert sch.peak_used <= 8 << 30


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_cooperative_run_matches_graph_run_bitwise(precision):
    """All steps in one cooperative launch (grid barrier between steps) give the
    bits of the graph of one launch per step, states and moments, over two runs."""
    import paper_1111_0922_amd as P
    K = 9
    out = {}
    for mode in ("graph", "cooperative"):
        batch = P.Batch(8, 4096, precision, mode=mode)
        grids = []
        for i, gm in enumerate(GEOMS):
            grid, _ = _grid(*gm, precision)
            if i == 2:
                grid.step(1)            # a slot at the other parity
            grids.append((batch.add(grid), grid))
        for _ in range(2):
            m = batch.run(K)
        out[mode] = ([from_device(g.get_pdfs()) for _, g in grids], [m[s].copy() for s, _ in grids],
                     [g.t for _, g in grids])
    for a, b in zip(out["graph"][0], out["cooperative"][0]):
        assert np.array_equal(a.view(np.int64), b.view(np.int64))
    for a, b in zip(out["graph"][1], out["cooperative"][1]):
        assert np.array_equal(a.view(np.int64), b.view(np.int64))
    assert out["graph"][2] == out["cooperative"][2]


def test_empty_batch_runs_and_reports_nothing():
    """A run with no active slot launches and returns; a slot added afterwards starts cleanly."""
    import paper_1111_0922_amd as P
    batch = P.Batch(4, 256, "f32")
    batch.run(4)                                  # no slot at all
    grid, _ = _grid(*GEOMS[0], "f32")
    s = batch.add(grid)
    batch.remove(s)
    batch.run(4)                                  # its only slot removed again
    assert grid.t == 0
    s = batch.add(grid)
    m = batch.run(6)
    ref, _ = _grid(*GEOMS[0], "f32")
    ref.step(6)
    assert np.array_equal(from_device(grid.get_pdfs()).view(np.int64), from_device(ref.get_pdfs()).view(np.int64))
    assert np.array_equal(m[s], from_device(ref.moments()))


def _poison(grid, node=7):
    """Replaces one node's canonical PDFs by NaN (a diverged lattice)."""
    f = grid.get_pdfs()
    f[:, node] = float("nan")
    grid.set_pdfs(f)


def test_diverged_slot_is_reported_alone_and_batch_mates_continue():
    """A lattice with a NaN node: lbm_batch_sync returns LBM_E_DIVERGED and marks that slot only; the
    other slots keep the bits they have alone, before and after the diverged one leaves."""
    import paper_1111_0922_amd as P
    from paper_1111_0922_amd.grid import _stream
    K = 10
    batch = P.Batch(8, 4096, "f32")
    grids = [_grid(*gm, "f32")[0] for gm in GEOMS]
    _poison(grids[2])
    slots = [batch.add(g) for g in grids]
    batch.run_async(K)
    status = np.zeros(batch.max_slots, dtype=np.int32)
    import ctypes
    rc = batch.lib.lbm_batch_sync(batch._h, ctypes.c_void_p(status.ctypes.data), _stream(batch.device))
    assert rc == P._lib.LBM_E_DIVERGED
    assert f"{slots[2]}".encode() in batch.lib.lbm_last_error()
    assert [int(status[s]) for s in slots] == [0, 0, 1, 0]
    m = batch.moments_host.numpy().copy()
    assert not np.isfinite(m[slots[2]]).all()
    batch.remove(slots[2])
    m2 = batch.run(K)
    assert not batch.last_status.any()
    for i in (0, 1, 3):
        ref = _grid(*GEOMS[i], "f32")[0]
        ref.step(K)
        assert np.array_equal(m[slots[i]], from_device(ref.moments()))
        ref.step(K)
        assert np.array_equal(m2[slots[i]], from_device(ref.moments()))
        assert np.array_equal(from_device(grids[i].get_pdfs()).view(np.int64), from_device(ref.get_pdfs()).view(np.int64))


def test_alone_equals_mix_with_a_192cube_request():
    """The largest serving lattice (192^3, request seed 7008) in a mix with smaller ones: every lattice
    ends with the bits it has alone (FP32, graph runs, two runs of K steps)."""
    import paper_1111_0922_amd as P

    def serving_grid(seed):
        mask, p = lbm_inputs.serving_geometry(seed)
        e = p["edge"]
        grid = P.Grid(e, e, e, addressing="indirect", precision="f32", omega=1.0, g=(1e-6, 0, 0), f16_scale=1024.0)
        grid.build_idx(torch.from_numpy(mask).cuda())
        grid.bind("aa")
        grid.init_equilibrium()
        return grid, e

    seeds = (7008, 7004, 7030, 7001)
    K = 50
    alone = []
    for s in seeds:
        grid, e = serving_grid(s)
        grid.step(2 * K)
        alone.append((from_device(grid.get_pdfs()), from_device(grid.moments()), e))
        del grid
    assert alone[0][2] == 192
    batch = P.Batch(8, 1 << 16, "f32")
    mix = [serving_grid(s)[0] for s in seeds]
    slots = [batch.add(g) for g in mix]
    for _ in range(2):
        m = batch.run(K)
    for s, g, (f, mo, _) in zip(slots, mix, alone):
        assert np.array_equal(from_device(g.get_pdfs()).view(np.int64), f.view(np.int64)), s
        assert np.array_equal(m[s].view(np.int64), mo.view(np.int64)), s


def test_scheduler_on_gpu_fails_only_the_diverged_request():
    """Served on the GPU executor, a request whose lattice is poisoned at admission ends as diverged;
    the others reach a steady state with the permeability they reach when served without it."""
    from paper_1111_0922_amd.serve import GpuExecutor, Request, Scheduler

    class Poisoning(GpuExecutor):
        def admit(self, req):
            super().admit(req)
            if req.seed == 7006:
                _poison(self.joining[req.rid])
                torch.cuda.synchronize()

    def serve(ex_cls, seeds):
        ex = ex_cls(max_slots=4, max_tiles=1 << 14, precision="f32")
        sch = Scheduler(ex, hbm_budget=8 << 30, max_slots=4, k_steps=100, tol=1e-6, max_steps=6000, prep_threads=2)
        out = sch.serve([Request(rid=i, seed=s, arrival=0.01 * i) for i, s in enumerate(seeds)])
        return {r.seed: r for r in out}, sch

    ref, _ = serve(GpuExecutor, (7004, 7039))
    got, sch = serve(Poisoning, (7004, 7006, 7039))
    assert got[7006].status == "diverged" and got[7006].steps == 100
    for s in (7004, 7039):
        assert got[s].status == ref[s].status and got[s].steps == ref[s].steps
        assert got[s].permeability == ref[s].permeability
    rep = sch.report(list(got.values()))
    assert rep["diverged"] == 1 and rep["requests"] == 3


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_rank_and_idx_slots_in_one_batch(precision):
    """A slot takes its grid's neighbour-id lookup (by rank by default, IDX when the option is off at
    lbm_batch_add); slots of both kinds in one batch reach the bits of the lattice run alone with IDX."""
    import paper_1111_0922_amd as P
    K = 15
    alone = []
    for gm in GEOMS[:3]:
        grid, _ = _grid(*gm, precision)
        grid.set_option(P._lib.OPT_RANK_LOOKUP, 0)
        grid.step(2 * K)
        alone.append(from_device(grid.get_pdfs()))
        del grid
    batch = P.Batch(8, 4096, precision, use_graph=True)
    grids = []
    for i, gm in enumerate(GEOMS[:3]):
        grid, _ = _grid(*gm, precision)
        grid.set_option(P._lib.OPT_RANK_LOOKUP, i % 2)
        assert grid.rank_lookup == bool(i % 2)
        grids.append((batch.add(grid), grid))
    for _ in range(2):
        batch.run(K)
    for (slot, grid), f_alone in zip(grids, alone):
        assert np.array_equal(from_device(grid.get_pdfs()).view(np.int64), f_alone.view(np.int64)), slot
