"""Neighbour ids by rank (LBM_OPT_RANK_LOOKUP): the arrays lbm_build_idx writes for it, and the same
bits as IDX in every kernel that reads neighbour ids.

With fluid ids in lexicographic order, the id of a fluid cell is the number of fluid cells before it.
The library stores, after the IDX rows and the slab block order, the cell of every node (cell_of) and
per 32 cells a pair (fluid bits, rank of the word's first fluid cell); the kernels then compute the 18
neighbour ids instead of reading IDX.  The arrays are compared entry by entry with the oracle's
numbering, and every update, read-out and reduction with the lookup on with the same calls with it off
and with the oracle.
"""
import numpy as np
import pytest
import torch

import lbm_inputs
import oracle
from lbm_cases import from_device, make_grid, to_device

pytestmark = pytest.mark.gpu


def _rank_arrays(grid):
    """(cell_of uint32[N_f], words uint32[n_words, 2]) read from the grid's IDX buffer."""
    s = grid.sizes("aa")
    nb = (grid.n_nodes + 255) // 256
    off = 18 * s.idx_pitch + (nb * 4 + 255) // 256 * 64          # int32 entries before cell_of
    flat = grid.idx.view(-1)
    cell_of = flat[off: off + grid.n_nodes].cpu().numpy().view(np.uint32)
    nw = (s.n_cells + 31) // 32
    w0 = off + s.idx_pitch
    words = flat[w0: w0 + 2 * nw].cpu().numpy().view(np.uint32).reshape(nw, 2)
    return cell_of, words


@pytest.mark.parametrize("shape,r,phi,seed", [((40, 37, 33), 4, 0.5, 1), ((64, 32, 16), 5, 0.45, 2),
                                              ((7, 1, 45), 1, 0.5, 3), ((33, 17, 5), 2, 0.6, 4)])
def test_rank_arrays_follow_the_oracle_numbering(shape, r, phi, seed):
    """cell_of[n] is the cell of fluid id n; word w has bit k set iff cell 32 w + k is fluid and holds
    the fluid id of its first fluid cell (0 when it has none).  Box sizes not divisible by 32 leave a
    ragged last word."""
    solid = lbm_inputs.sphere_pack(shape, r, phi, seed=seed)[0]
    grid = make_grid(solid, "aa", addressing="indirect")
    cm, _, nf = oracle.build_idx(solid, with_idx=False)
    assert grid.n_nodes == nf
    cell_of, words = _rank_arrays(grid)
    assert np.array_equal(cell_of.astype(np.int64), oracle.node_order(cm))
    flat = solid.reshape(-1)
    nw = words.shape[0]
    pad = np.zeros(32 * nw, np.uint8)
    pad[: flat.size] = flat == 0
    fluid = pad.reshape(nw, 32).astype(np.uint64)
    bits = (fluid << np.arange(32, dtype=np.uint64)).sum(axis=1)
    assert np.array_equal(words[:, 0].astype(np.uint64), bits)
    cmf = np.concatenate([cm.reshape(-1), np.full(32 * nw - flat.size, -1, np.int32)]).reshape(nw, 32)
    has = fluid.any(axis=1)
    first = np.argmax(fluid, axis=1)
    want_rank = np.where(has, cmf[np.arange(nw), first], 0)
    assert np.array_equal(words[:, 1].astype(np.int64), want_rank.astype(np.int64))


OFFS = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1)]


@pytest.mark.parametrize("shape,r,phi,seed", [((40, 37, 33), 4, 0.5, 1), ((7, 1, 45), 1, 0.5, 3)])
def test_ghost_words_follow_the_ghost_numbering(shape, r, phi, seed):
    """With et_ghosts, the ghost words after the rank words: bit k of word w set iff cell 32 w + k is a
    ghost (a solid cell s with s - o fluid for one of the esoteric twist's six offsets o), and the ghost
    number of the word's first ghost (ghosts numbered in lexicographic order)."""
    solid = lbm_inputs.sphere_pack(shape, r, phi, seed=seed)[0]
    grid = make_grid(solid, "et", addressing="indirect")
    s = grid.sizes("et")
    nb = (grid.n_nodes + 255) // 256
    nw = (s.n_cells + 31) // 32
    off = 18 * s.idx_pitch + (nb * 4 + 255) // 256 * 64 + s.idx_pitch + (nw * 8 + 255) // 256 * 64
    words = grid.idx.view(-1)[off: off + 2 * nw].cpu().numpy().view(np.uint32).reshape(nw, 2)
    fluid = solid == 0
    ghost = np.zeros_like(fluid)
    for o in OFFS:
        ghost |= (solid != 0) & np.roll(fluid, (o[2], o[1], o[0]), axis=(0, 1, 2))
    assert int(ghost.sum()) == s.n_ghost
    g = np.zeros(32 * nw, np.uint64)
    g[: solid.size] = ghost.reshape(-1)
    g = g.reshape(nw, 32)
    assert np.array_equal(words[:, 0].astype(np.uint64), (g << np.arange(32, dtype=np.uint64)).sum(axis=1))
    before = np.concatenate([[0], np.cumsum(g.sum(axis=1))[:-1]]).astype(np.int64)
    want = np.where(g.any(axis=1), before, 0)
    assert np.array_equal(words[:, 1].astype(np.int64), want)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("layout", ["soa", "aos"])
@pytest.mark.parametrize("scheme", ["aa", "ts", "os_push", "os_pull", "et"])
def test_rank_lookup_gives_the_idx_bits(scheme, layout, precision):
    """7 steps (AA and ET end in their odd-t state, read out through the gathering map), moments
    included; the esoteric twist takes its storage addresses and solid mask from the same words."""
    import paper_1111_0922_amd as P
    solid = lbm_inputs.sphere_pack((45, 38, 29), 4, 0.55, seed=51)[0]
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=52))
    f0 = oracle.fluid_view(oracle.init_equilibrium(ru, solid), solid)
    grid = make_grid(solid, scheme, addressing="indirect", layout=layout, precision=precision, omega=1.3,
                     g=(1e-5, 2e-6, 0))
    out = []
    for rank in (0, 1):
        grid.set_option(P._lib.OPT_RANK_LOOKUP, rank)
        assert grid.rank_lookup == bool(rank) and grid.et_rank_lookup == bool(rank and scheme == "et")
        grid.set_pdfs(to_device(f0))
        grid.step(7)
        out.append((from_device(grid.get_pdfs()), from_device(grid.moments())))
    assert np.array_equal(out[0][0].view(np.int64), out[1][0].view(np.int64))
    assert np.array_equal(out[0][1], out[1][1])
    if precision == "f64":
        want = oracle.fluid_view(oracle.run_ts(oracle.init_equilibrium(ru, solid), solid, 7, 1.3, (1e-5, 2e-6, 0)),
                                 solid)
        assert float(np.max(np.abs(out[1][0] - want) / np.abs(want))) <= 1e-12


@pytest.mark.parametrize("scheme", ["aa", "os_pull"])
def test_rank_lookup_with_a_caller_block_order_and_trt(scheme):
    import paper_1111_0922_amd as P
    solid = lbm_inputs.sphere_pack((50, 40, 30), 4, 0.5, seed=53)[0]
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=54))
    f0 = oracle.fluid_view(oracle.init_equilibrium(ru, solid), solid)
    grid = make_grid(solid, scheme, addressing="indirect", omega=1.5, g=(1e-5, 0, 0))
    nb = (grid.n_nodes + 255) // 256
    out = []
    for rank in (0, 1):
        grid.set_option(P._lib.OPT_RANK_LOOKUP, rank)
        grid.set_block_order(torch.from_numpy(np.random.default_rng(rank).permutation(nb).astype(np.int32)).cuda())
        grid.set_pdfs(to_device(f0))
        grid.step(5, collider="trt")
        out.append(from_device(grid.get_pdfs()))
    assert np.array_equal(out[0].view(np.int64), out[1].view(np.int64))


def test_rank_lookup_is_ignored_with_open_boundaries_and_bricks():
    """Open-boundary classes need IDX's class codes and bricked numberings are not ranks: the option
    then changes nothing (and bricked grids store no rank arrays)."""
    import paper_1111_0922_amd as P
    duct = np.zeros((12, 10, 24), np.uint8)
    duct[:, :, 0] = 2
    duct[:, :, -1] = 3
    duct[0] = duct[-1] = 1
    out = []
    for rank in (0, 1):
        grid = make_grid(duct, "aa", addressing="indirect", omega=1.2)
        grid.set_boundary(1, "velocity", 1.0, (0.01, 0, 0))
        grid.set_boundary(2, "pressure", 1.0, (0.0, 0, 0))
        grid.set_option(P._lib.OPT_RANK_LOOKUP, rank)
        grid.init_equilibrium()
        grid.step(9)
        out.append(from_device(grid.get_pdfs()))
    assert np.array_equal(out[0].view(np.int64), out[1].view(np.int64))
    solid = lbm_inputs.sphere_pack((32, 24, 16), 3, 0.5, seed=55)[0]
    sizes = []
    out = []
    for rank, brick in ((0, None), (1, (8, 8, 8))):
        grid = make_grid(solid, "aa", addressing="indirect", brick=brick)
        grid.set_option(P._lib.OPT_RANK_LOOKUP, rank)
        grid.init_equilibrium()
        grid.step(4)
        sizes.append(grid.sizes("aa").idx_bytes)
        out.append((grid.cellmap[: solid.size].cpu().numpy(), from_device(grid.get_pdfs())))
    assert sizes[1] < sizes[0]   # no cell_of / rank words for the bricked numbering
    # the same state cell by cell
    (cm0, f0), (cm1, f1) = out
    fl = cm0 >= 0
    assert np.array_equal(f0[:, cm0[fl]].view(np.int64), f1[:, cm1[fl]].view(np.int64))


def test_build_call_two_requires_the_mask():
    """The fill pass reads the boundary classes (and the rank words the fluid bits) from the mask."""
    import ctypes
    import paper_1111_0922_amd as P
    L = P._lib
    solid = lbm_inputs.sphere_pack((16, 16, 16), 3, 0.5, seed=56)[0]
    grid = make_grid(solid, "aa", addressing="indirect")
    s = grid.sizes("aa")
    scratch = torch.empty(s.build_scratch_bytes, dtype=torch.uint8, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    nf = ctypes.c_int64(0)
    rc = grid.lib.lbm_build_idx(grid._h, None, p(grid.cellmap), p(grid.idx), None, p(scratch), ctypes.byref(nf), None)
    assert rc == L.LBM_E_ARG
    assert "d_mask" in grid.lib.lbm_last_error().decode()
