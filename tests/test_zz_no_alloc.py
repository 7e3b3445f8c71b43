"""lbm_reduce_moments_noalloc (the moment reduction that allocates nothing) against lbm_reduce_moments.

Both run the same reduction kernels; the entry point without allocation only
keeps its per-block partials in the library's static device array instead of
the grid's bound scratch.  So the two must agree bit for bit, on every call,
including a second call on a smaller lattice after a larger one (the array
then still holds the larger lattice's partials beyond the smaller one's).
"""
import ctypes

import numpy as np
import pytest
import torch

import lbm_inputs
import oracle
from lbm_cases import from_device, make_grid, to_device


def _pair(grid):
    """(existing entry point, entry point without allocation), both as float64[4] on the host."""
    want = grid.moments()
    got = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    grid.moments_noalloc(got)
    return from_device(want), from_device(got)


@pytest.mark.gpu
def test_noalloc_moments_match_bound_scratch_twice_then_smaller():
    # call 1: indirect FP64 sphere pack after an odd number of AA steps (the odd-step read map)
    solid = lbm_inputs.sphere_pack(48, 5, 0.55, seed=21)[0]
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=22))
    f0 = oracle.init_equilibrium(ru, solid)
    big = make_grid(solid, "aa", addressing="indirect", omega=1.3, g=(1e-5, 0.0, 2e-6))
    big.set_pdfs(to_device(oracle.fluid_view(f0, solid)))
    big.step(3)
    want, got = _pair(big)
    assert np.array_equal(want.view(np.int64), got.view(np.int64)), (want, got)
    # the oracle's own moments of the same state (FP64, 1e-12 as every FP64 parity bar)
    ref = oracle.moments(oracle.run_ts(f0, solid, 3, 1.3, (1e-5, 0.0, 2e-6)), solid)
    assert abs(got[0] - ref[0]) / abs(ref[0]) <= 1e-12
    assert np.max(np.abs(got[1:] - ref[1:])) <= 1e-12 * abs(ref[0])
    # call 2, right after: a smaller lattice (fewer blocks), other storage, layout and scheme
    small = make_grid(lbm_inputs.channel_mask(16, 12, 10), "os_pull", layout="aos", precision="f32",
                      omega=1.0, g=(1e-6, 0.0, 0.0))
    small.init_equilibrium()
    small.step(5)
    want2, got2 = _pair(small)
    assert np.array_equal(want2.view(np.int64), got2.view(np.int64)), (want2, got2)
    assert big.n_nodes > 4 * small.n_nodes
    # call 3: the larger lattice again, one step on; still the same bits
    big.step(1)
    want3, got3 = _pair(big)
    assert np.array_equal(want3.view(np.int64), got3.view(np.int64)), (want3, got3)


@pytest.mark.gpu
def test_noalloc_moments_at_the_size_limit_boundary():
    """A direct grid one row under the static limit is served, with the same bits as the bound scratch."""
    import paper_1111_0922_amd as P
    n_max = P._lib.NOALLOC_MAX_NODES
    grid = P.Grid(1024, 256, 256, precision="f16s", wall_z=False, omega=1.0, f16_scale=1024.0)
    assert grid.n_nodes == n_max
    grid.bind("aa")
    grid.init_equilibrium()
    grid.step(1)
    want, got = _pair(grid)
    assert np.array_equal(want.view(np.int64), got.view(np.int64)), (want, got)
    assert abs(got[0] - n_max) / n_max <= 1e-6


def test_noalloc_rejects_oversized_grid_without_gpu():
    """More nodes than the static array covers: LBM_E_ARG before any device work (runs on the CPU)."""
    import paper_1111_0922_amd as P
    L = P._lib
    grid = P.Grid(512, 512, 259, wall_z=True)       # 512 * 512 * 257 nodes > 2^26
    assert grid.n_nodes > L.NOALLOC_MAX_NODES
    out = np.zeros(4)
    rc = grid.lib.lbm_reduce_moments_noalloc(grid._h, ctypes.c_void_p(out.ctypes.data), None)
    assert rc == L.LBM_E_ARG
    assert b"static" in grid.lib.lbm_last_error()
    # an unbound grid within the limit: LBM_E_STATE, also before any device work
    small = P.Grid(8, 8, 8)
    assert small.lib.lbm_reduce_moments_noalloc(small._h, ctypes.c_void_p(out.ctypes.data), None) == L.LBM_E_STATE
    assert small.lib.lbm_reduce_moments_noalloc(small._h, None, None) == L.LBM_E_ARG
