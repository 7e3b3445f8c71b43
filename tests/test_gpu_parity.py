"""FP64 parity of every GPU scheme against the FP64 oracle (two-step, pull).

Bars (from the build's stated targets): FP64 node values within 1e-12
relative of the oracle after 100 steps of the 32^3 channel; mass conserved
to 1e-13; all schemes, layouts and addressings bit-identical to each other
at even step counts (they share one collision and only move bits otherwise).
"""
import numpy as np
import pytest
import torch

import lbm_inputs
import oracle
from lbm_cases import (ADDRESSING, LAYOUTS, SCHEMES, config1, dense_from_canon, from_device, make_grid, rel_err,
                       to_device)

pytestmark = pytest.mark.gpu

STEPS = 100


@pytest.fixture(scope="module")
def oracle_config1():
    solid, f0, omega, g = config1()
    f100 = oracle.run_ts(f0, solid, STEPS, omega, g)
    return solid, f0, f100, omega, g


@pytest.fixture(scope="module")
def gpu_results():
    return {}


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("addressing", ADDRESSING)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_fp64_config1_matches_oracle(scheme, addressing, layout, oracle_config1, gpu_results):
    solid, f0, f100, omega, g = oracle_config1
    grid = make_grid(solid, scheme, addressing=addressing, layout=layout, omega=omega, g=g)
    grid.set_pdfs(to_device(oracle.fluid_view(f0, solid)))
    m0 = from_device(grid.moments())
    grid.step(STEPS)
    got = from_device(grid.get_pdfs())
    want = oracle.fluid_view(f100, solid)
    assert rel_err(got, want) <= 1e-12
    m1 = from_device(grid.moments())
    assert abs(m1[0] - m0[0]) / m0[0] <= 1e-13
    mo = oracle.moments(f100, solid)
    assert abs(m1[0] - mo[0]) / mo[0] <= 1e-13
    np.testing.assert_allclose(m1[1:], mo[1:], rtol=1e-9, atol=1e-13 * mo[0])
    gpu_results[(scheme, addressing, layout)] = got


@pytest.mark.parametrize("block", [0, 4096])
def test_fp64_config1_direct_aa_plain_and_blocked(block, oracle_config1, gpu_results):
    """The direct AA pattern in plain SoA (the paper's layout, which the benchmark's headline runs) and
    in 4096-cell blocks (the default for FP64 lattices whose rows fit whole blocks) against the oracle."""
    import paper_1111_0922_amd as P
    solid, f0, f100, omega, g = oracle_config1
    grid = make_grid(solid, "aa", omega=omega, g=g)
    assert grid.lattice_block == 4096
    grid.set_option(P._lib.OPT_SOA_BLOCK, block)
    grid.bind("aa")
    assert grid.lattice_block == block
    grid.set_pdfs(to_device(oracle.fluid_view(f0, solid)))
    grid.step(STEPS)
    got = from_device(grid.get_pdfs())
    assert rel_err(got, oracle.fluid_view(f100, solid)) <= 1e-12
    gpu_results[("aa", "direct", f"soa_block{block}")] = got


def test_all_variants_bit_identical(gpu_results):
    """Propagation only moves bits and all kernels share one collision: identical states."""
    keys = sorted(gpu_results)
    if len(keys) < 2:
        pytest.skip("needs the parity runs of this module")
    ref = gpu_results[keys[0]]
    for k in keys[1:]:
        assert np.array_equal(gpu_results[k].view(np.int64), ref.view(np.int64)), k


@pytest.mark.parametrize("scheme", SCHEMES)
def test_odd_step_counts_match_oracle(scheme):
    """Odd t exercises the AA odd-step readout and the esoteric twist's odd parity."""
    solid, f0, omega, g = config1()
    f7 = oracle.run_ts(f0, solid, 7, 1.6, g)
    for addressing in ADDRESSING:
        grid = make_grid(solid, scheme, addressing=addressing, omega=1.6, g=g)
        grid.set_pdfs(to_device(oracle.fluid_view(f0, solid)))
        grid.step(7)
        assert rel_err(from_device(grid.get_pdfs()), oracle.fluid_view(f7, solid)) <= 1e-13


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("shape", [(11, 5, 37), (3, 1, 1), (4, 3, 2)])
def test_ragged_periodic_boxes(scheme, shape):
    """Box sizes that are not powers of two, node counts off the 256-lane blocks, axes of length 1."""
    solid = np.zeros(shape, np.uint8)
    ru = lbm_inputs.rho_u_field(shape, lbm_inputs.velocity_noise(shape, 1e-2, seed=4))
    f0 = oracle.init_equilibrium(ru, solid)
    g = (1e-5, -3e-5, 2e-5)
    want = oracle.fluid_view(oracle.run_ts(f0, solid, 10, 1.3, g), solid)
    for addressing in ADDRESSING:
        for layout in LAYOUTS:
            grid = make_grid(solid, scheme, addressing=addressing, layout=layout, omega=1.3, g=g)
            grid.set_pdfs(to_device(oracle.fluid_view(f0, solid)))
            grid.step(10)
            assert rel_err(from_device(grid.get_pdfs()), want) <= 1e-13, (addressing, layout)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("layout", LAYOUTS)
def test_porous_indirect_matches_oracle(scheme, layout):
    solid = lbm_inputs.sphere_pack((29, 21, 18), 3, 0.5, seed=6)[0]
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=5))
    f0 = oracle.init_equilibrium(ru, solid)
    g = (1e-5, 0, 0)
    want = oracle.fluid_view(oracle.run_ts(f0, solid, 40, 1.6, g), solid)
    grid = make_grid(solid, scheme, addressing="indirect", layout=layout, omega=1.6, g=g)
    grid.set_pdfs(to_device(oracle.fluid_view(f0, solid)))
    grid.step(40)
    assert rel_err(from_device(grid.get_pdfs()), want) <= 1e-12


@pytest.mark.parametrize("addressing", ADDRESSING)
def test_init_equilibrium_matches_oracle(addressing):
    solid, _, _, _ = config1()
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-2, seed=8))
    ru[0] += 0.01 * lbm_inputs.uniform01(9, solid.size).reshape(solid.shape)
    want = oracle.fluid_view(oracle.init_equilibrium(ru, solid), solid)
    rho_u = ru.reshape(4, -1)[:, solid.reshape(-1) == 0]
    for scheme in SCHEMES:
        grid = make_grid(solid, scheme, addressing=addressing)
        grid.init_equilibrium(to_device(rho_u))
        got = from_device(grid.get_pdfs())
        assert float(np.max(np.abs(got - want))) <= 1e-15


def test_rest_init_and_rest_fixed_point():
    solid = lbm_inputs.channel_mask(8, 8, 8)
    want = oracle.fluid_view(oracle.init_equilibrium(lbm_inputs.rho_u_field(solid.shape), solid), solid)
    for scheme in SCHEMES:
        grid = make_grid(solid, scheme, omega=1.4)
        grid.init_equilibrium()
        np.testing.assert_array_equal(from_device(grid.get_pdfs()), want)
        grid.step(10)
        assert float(np.max(np.abs(from_device(grid.get_pdfs()) - want))) <= 2e-16


def test_reduction_deterministic_and_matches_canonical_sums():
    solid, f0, omega, g = config1()
    grid = make_grid(solid, "aa", omega=omega, g=g)
    grid.set_pdfs(to_device(oracle.fluid_view(f0, solid)))
    grid.step(3)
    a = from_device(grid.moments())
    b = from_device(grid.moments())
    assert np.array_equal(a, b)
    canon = from_device(grid.get_pdfs())
    c = np.array([[0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0],
                  [0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1],
                  [0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1]])
    want = np.concatenate([[np.sum(canon, dtype=np.float64)], (c @ canon).sum(axis=1)])
    np.testing.assert_allclose(a, want, rtol=1e-12, atol=1e-15)


def test_nan_shows_in_mass():
    solid = lbm_inputs.channel_mask(8, 8, 8)
    grid = make_grid(solid, "aa")
    grid.init_equilibrium()
    canon = grid.get_pdfs()
    canon[3, 17] = float("nan")
    grid.set_pdfs(canon)
    assert np.isnan(from_device(grid.moments())[0])


def test_scheme_mismatch_is_an_error():
    import paper_1111_0922_amd as P
    solid = lbm_inputs.channel_mask(8, 8, 8)
    grid = make_grid(solid, "aa")
    # refused before any launch
    assert grid.lib.lbm_step(grid._h, P._lib.ET, P._lib.BGK, 1, None) == P._lib.LBM_E_STATE


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("shape", [(32, 32, 32), (6, 5, 64), (5, 3, 256), (4, 4, 2), (5, 3, 512), (4, 2, 768),
                                   (4, 3, 384), (3, 3, 257), (5, 4, 100), (7, 5, 6)])
def test_row_staged_kernels_bit_identical_to_plain(scheme, shape):
    """Direct SoA grids run row-staged kernels (whole rows, row segments, or rows spanning
    workgroups for any other nx); the plain kernels must agree bit for bit.  Shapes are (nz, ny, nx)."""
    import paper_1111_0922_amd as P
    solid = lbm_inputs.channel_mask(shape[2], shape[1], shape[0])
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-2, seed=12))
    f0 = oracle.fluid_view(oracle.init_equilibrium(ru, solid), solid)
    out = []
    for staged in (1, 0):
        grid = make_grid(solid, scheme, omega=1.7, g=(1e-5, 2e-5, 0))
        grid.set_option(P._lib.OPT_ROW_STAGE, staged)
        grid.set_pdfs(to_device(f0))
        grid.step(5)
        out.append(from_device(grid.get_pdfs()))
    assert np.array_equal(out[0].view(np.int64), out[1].view(np.int64))
    want = oracle.fluid_view(oracle.run_ts(dense_from_canon(f0, solid), solid, 5, 1.7, (1e-5, 2e-5, 0)), solid)
    assert rel_err(out[0], want) <= 1e-13


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("brick", [(4, 4, 4), (8, 2, 4)])
def test_brick_ordered_indirect_matches_oracle(scheme, brick):
    """Fluid ids in brick order: the canonical node order is the grid's id order."""
    solid = lbm_inputs.sphere_pack((29, 21, 18), 3, 0.5, seed=6)[0]
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=5))
    f0 = oracle.init_equilibrium(ru, solid)
    g = (1e-5, 0, 0)
    cellmap, _, nf = oracle.build_idx(solid, brick=brick)
    order = oracle.node_order(cellmap)
    want = oracle.ordered_view(oracle.run_ts(f0, solid, 21, 1.6, g), order)
    grid = make_grid(solid, scheme, addressing="indirect", omega=1.6, g=g, brick=brick)
    grid.set_pdfs(to_device(oracle.ordered_view(f0, order)))
    grid.step(21)
    assert rel_err(from_device(grid.get_pdfs()), want) <= 1e-12


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("shape,precision", [((256, 32, 6), "f64"), ((64, 64, 5), "f64"), ((512, 16, 4), "f16s")])
def test_banded_block_order_bit_identical(scheme, layout, shape, precision):
    """The XCD band order only permutes which workgroup updates which nodes."""
    import paper_1111_0922_amd as P
    solid = lbm_inputs.channel_mask(shape[0], shape[1], shape[2])
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=14))
    f0 = oracle.fluid_view(oracle.init_equilibrium(ru, solid), solid)
    out = []
    for band in (0, -1, 1, 2, 4):
        grid = make_grid(solid, scheme, layout=layout, precision=precision, omega=1.7, g=(1e-5, 0, 0))
        grid.set_option(P._lib.OPT_BAND, band)
        grid.set_pdfs(to_device(f0))
        grid.step(5)
        out.append(from_device(grid.get_pdfs()))
    for o in out[1:]:
        assert np.array_equal(o.view(np.int64), out[0].view(np.int64))



@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("addressing,layout", [("direct", "soa"), ("direct", "aos"), ("indirect", "soa"),
                                               ("indirect", "aos")])
def test_layout_and_launch_options_bit_identical(scheme, addressing, layout):
    """Pitch padding, the LDS reservation (residency) and the XCD-aware block order change
    addresses and launch shapes only: every setting gives the same bits."""
    import paper_1111_0922_amd as P
    L = P._lib
    if addressing == "direct":
        solid = lbm_inputs.channel_mask(32, 10, 9)
    else:
        solid = lbm_inputs.sphere_pack((20, 14, 12), 3, 0.6, 41)[0]
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-2, seed=42))
    f0 = oracle.fluid_view(oracle.init_equilibrium(ru, solid), solid)
    settings = [{}, {L.OPT_PITCH_PAD: 33920}, {L.OPT_WG_LDS: 0}, {L.OPT_WG_LDS: 98304}, {L.OPT_XCD_REMAP: 1}]
    out = []
    for opts in settings:
        grid = make_grid(solid, scheme, addressing=addressing, layout=layout, omega=1.7, g=(1e-5, 2e-5, 0))
        for k, v in opts.items():
            grid.set_option(k, v)
        grid.bind(scheme)  # the pitch pad changes the buffer sizes
        grid.set_pdfs(to_device(f0))
        grid.step(5)
        out.append((from_device(grid.get_pdfs()), from_device(grid.moments())))
    for f, m in out[1:]:
        assert np.array_equal(f.view(np.int64), out[0][0].view(np.int64))
        assert np.array_equal(m.view(np.int64), out[0][1].view(np.int64))


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("nx,precision", [(300, "f64"), (512, "f64"), (384, "f16s"), (1024, "f16s")])
def test_launch_options_bit_identical_on_wide_rows(scheme, nx, precision):
    """The kernels across rows (nx = 300, 384), on row segments (512) and with two nodes per lane
    on row segments (FP16, 1024) under the XCD-aware block order, the LDS reservation and pitch
    padding: the same bits."""
    import paper_1111_0922_amd as P
    L = P._lib
    solid = lbm_inputs.channel_mask(nx, 3, 5)
    sigma = 64.0 if precision == "f16s" else 1.0
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-2, seed=43))
    f0 = oracle.fluid_view(oracle.init_equilibrium(ru, solid), solid)
    settings = [{}, {L.OPT_XCD_REMAP: 1}, {L.OPT_WG_LDS: 0}, {L.OPT_WG_LDS: 65536}, {L.OPT_PITCH_PAD: 4224}]
    out = []
    for opts in settings:
        grid = make_grid(solid, scheme, precision=precision, omega=1.7, g=(1e-5, 2e-5, 0), f16_scale=sigma)
        for k, v in opts.items():
            grid.set_option(k, v)
        grid.bind(scheme)
        grid.set_pdfs(to_device(f0))
        grid.step(5)
        out.append(from_device(grid.get_pdfs()))
    for f in out[1:]:
        assert np.array_equal(f.view(np.int64), out[0].view(np.int64))
