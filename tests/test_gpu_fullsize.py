"""Parity at the benchmark sizes, in the launch configuration the benchmark times.

The oracle cannot run 256^3 or 512^3 lattices for many steps in a test, so
these checks use what it can compute one node at a time: from the GPU's
canonical state f(t), the oracle's own two-step update of each sampled node's
3x3x3 neighbourhood (non-periodic, so only the centre is complete) gives
f(t+1) at the centre, which must match the GPU's f(t+1) to 1e-12.  Mass
conservation and cross-scheme identity are checked on the whole lattice.
"""
import numpy as np
import pytest
import torch

import lbm_inputs
import oracle
from lbm_cases import from_device, make_grid, rel_err, to_device

pytestmark = pytest.mark.gpu


def _sample_update(canon_t, solid, cells, omega, g, **kw):
    """Oracle f(t+1) at `cells` (flat indices) from the canonical state f(t) (fluid nodes only);
    kw goes to oracle.run_ts (collider, precision, sigma, omega_minus, bc)."""
    nz, ny, nx = solid.shape
    ids = _fluid_ids(solid)
    out = []
    for c in cells:
        z, y, x = np.unravel_index(c, solid.shape)
        zi = [(z + d) % nz for d in (-1, 0, 1)]
        yi = [(y + d) % ny for d in (-1, 0, 1)]
        xi = [(x + d) % nx for d in (-1, 0, 1)]
        sub_cells = (np.array(zi)[:, None, None] * ny + np.array(yi)[None, :, None]) * nx + np.array(xi)[None, None, :]
        sub_s = solid.reshape(-1)[sub_cells]
        sub_ids = ids[sub_cells]
        sub_f = np.where(sub_ids >= 0, canon_t[:, np.maximum(sub_ids, 0)], 0.0)
        nxt = oracle.run_ts(sub_f, sub_s, 1, omega, g, periodic=(0, 0, 0), **kw)
        out.append(nxt[:, 1, 1, 1])
    return np.array(out).T


def _fluid_ids(solid):
    ids = np.full(solid.size, -1, np.int64)
    fl = solid.reshape(-1) == 0
    ids[fl] = np.arange(int(fl.sum()))
    return ids


@pytest.mark.parametrize("layout", ["soa", "aos"])
@pytest.mark.parametrize("scheme", ["ts", "os_push", "os_pull", "aa", "et"])
def test_256_channel_sampled(scheme, layout):
    """Every scheme x layout of the benchmark's table, at its size and in its launch configuration
    (row staging, residency, the AoS band order; the library's default storage order, which for the
    AA pattern in FP64 is 4096-cell blocks)."""
    _channel_sampled(scheme, layout)


def test_256_channel_sampled_aa_plain_soa():
    """The headline's configuration: the AA pattern on the 256^3 channel in plain SoA."""
    _channel_sampled("aa", "soa", block=0)


def _channel_sampled(scheme, layout, block=None):
    import paper_1111_0922_amd as P
    n = 256
    solid = lbm_inputs.channel_mask(n, n, n)
    omega, g = 1.6, (1e-6, 0.0, 0.0)
    rng = np.random.default_rng(1)
    grid = make_grid(solid, scheme, layout=layout, omega=omega, g=g)
    if block is not None:
        grid.set_option(P._lib.OPT_SOA_BLOCK, block)
        grid.bind(scheme)
        assert grid.lattice_block == block
    nf = grid.n_nodes
    u = torch.from_numpy(lbm_inputs.velocity_noise((n - 2, n, n), 1e-3, seed=1).reshape(3, -1))
    rho_u = torch.cat([torch.ones(1, nf, dtype=torch.float64), u], 0)
    grid.init_equilibrium(rho_u.cuda())
    m0 = from_device(grid.moments())
    grid.step(9)  # odd count: the next step runs the other kernel of the pair
    for extra in (1, 2):
        ft = from_device(grid.get_pdfs())
        grid.step(1)
        ft1 = from_device(grid.get_pdfs())
        cells = rng.choice(np.flatnonzero(solid.reshape(-1) == 0), 300, replace=False)
        cells = np.concatenate([cells, [n * n + 0, n * n * (n - 1) - 1, n * n + n - 1]])  # wrap corners
        ids = _fluid_ids(solid)[cells]
        want = _sample_update(ft, solid, cells, omega, g)
        assert rel_err(ft1[:, ids], want) <= 1e-12, extra
        del ft, ft1
    m1 = from_device(grid.moments())
    assert abs(m1[0] - m0[0]) / m0[0] <= 1e-13


@pytest.mark.parametrize("case", ["f16s", "f32", "f32s", "trt"])
def test_256_channel_sampled_precision_and_trt(case):
    """The benchmark's FP16 (two nodes per lane), FP32, FP32-shifted and TRT runs at full size, with
    the scale sigma = 1024 the benchmark gives the shifted forms.  The bars are the small-lattice
    precision tests', which hold while |f - w_i| < 2^-12 (checked on the state)."""
    n = 256
    solid = lbm_inputs.channel_mask(n, n, n)
    omega, g = 1.6, (1e-6, 0.0, 0.0)
    prec = case if case != "trt" else "f64"
    sigma = 1024.0 if prec in ("f16s", "f32s") else 1.0
    rng = np.random.default_rng(2)
    grid = make_grid(solid, "aa", precision=prec, omega=omega, g=g, f16_scale=sigma)
    if case == "trt":            # the benchmark runs TRT on the headline's plain SoA
        import paper_1111_0922_amd as P
        grid.set_option(P._lib.OPT_SOA_BLOCK, 0)
        grid.bind("aa")
    nf = grid.n_nodes
    u = torch.from_numpy(lbm_inputs.velocity_noise((n - 2, n, n), 1e-3, seed=1).reshape(3, -1))
    grid.init_equilibrium(torch.cat([torch.ones(1, nf, dtype=torch.float64), u], 0).cuda())
    collider = "trt" if case == "trt" else "bgk"
    kw = {"collider": collider}
    if case == "trt":
        kw["omega_minus"] = oracle.trt_omega_minus(omega, 3.0 / 16.0)
    if prec != "f64":
        kw.update(precision=prec, sigma=sigma)
    grid.step(9, collider=collider)
    for extra in (1, 2):
        ft = from_device(grid.get_pdfs())
        if prec != "f64":
            assert float(np.max(np.abs(ft - oracle.tables()[1][:, None]))) < 2.0 ** -12
        grid.step(1, collider=collider)
        ft1 = from_device(grid.get_pdfs())
        cells = rng.choice(np.flatnonzero(solid.reshape(-1) == 0), 300, replace=False)
        ids = _fluid_ids(solid)[cells]
        want = _sample_update(ft, solid, cells, omega, g, **kw)
        if prec == "f32s":       # the stored deviation carries 2^-24 of itself; FP32 arithmetic on it
            assert float(np.max(np.abs(ft1[:, ids] - want))) <= 2e-9, extra
        elif prec == "f16s":       # one binary16 code of h = (f - w) sigma may round the other way: 2^-23 in f
            assert float(np.max(np.abs(ft1[:, ids] - want))) <= 4 * 2.0 ** -23, extra
        elif prec == "f32":      # FP32 arithmetic of one collision: 16 ulp
            assert rel_err(ft1[:, ids], want) <= 1e-6, extra
        else:
            assert rel_err(ft1[:, ids], want) <= 1e-12, extra
        del ft, ft1


def test_256_duct_open_boundaries_sampled():
    """The benchmark's 256^3 duct (velocity inlet, pressure outlet, walls) at full size; the
    samples include nodes next to the inlet and the outlet."""
    n = 256
    duct = np.zeros((n, n, n), np.uint8)
    duct[:, :, 0] = 2
    duct[:, :, n - 1] = 3
    duct[0] = 1
    duct[n - 1] = 1
    bc = {1: ("velocity", 1.0, (0.01, 0.0, 0.0)), 2: ("pressure", 1.0, (0.01, 0.0, 0.0))}
    omega, g = 1.6, (0.0, 0.0, 0.0)
    grid = make_grid(duct, "aa", addressing="indirect", omega=omega, g=g)
    for cls, (kind, rho, u) in bc.items():
        grid.set_boundary(cls, kind, rho, u)
    grid.init_equilibrium()
    grid.step(9)
    rng = np.random.default_rng(3)
    fluid = np.flatnonzero(duct.reshape(-1) == 0)
    for extra in (1, 2):
        ft = from_device(grid.get_pdfs())
        grid.step(1)
        ft1 = from_device(grid.get_pdfs())
        edge = fluid[(fluid % n == 1) | (fluid % n == n - 2)]
        cells = np.concatenate([rng.choice(fluid, 200, replace=False), rng.choice(edge, 100, replace=False)])
        ids = _fluid_ids(duct)[cells]
        want = _sample_update(ft, duct, cells, omega, g, bc=bc)
        assert rel_err(ft1[:, ids], want) <= 1e-12, extra
        del ft, ft1


@pytest.fixture(scope="module")
def pack512():
    solid, count = lbm_inputs.sphere_pack(512, 8, 0.40, seed=3)
    return solid


@pytest.mark.parametrize("scheme", ["aa", "ts", "os_push", "os_pull", "et"])
def test_512_porous_sampled(scheme, pack512):
    """Every scheme of the benchmark's pack table, in its launch configuration (the XCD slab order
    of the kernels that write to neighbours); both kernels of AA and ET are sampled."""
    solid = pack512
    omega, g = 1.6, (1e-6, 0.0, 0.0)
    grid = make_grid(solid, scheme, addressing="indirect", omega=omega, g=g)
    cellmap_o, _, nf = oracle.build_idx(solid, with_idx=False)
    assert grid.n_nodes == nf
    cm = grid.cellmap[: solid.size]
    assert torch.equal(torch.where(cm >= 0, cm, torch.full_like(cm, -1)).cpu(),
                       torch.from_numpy(cellmap_o.reshape(-1)))
    grid.cellmap = None
    grid._mask = None
    grid.init_equilibrium()
    m0 = from_device(grid.moments())
    grid.step(3)
    rng = np.random.default_rng(2)
    ids_all = _fluid_ids(solid)
    for extra in (1, 2):
        ft = from_device(grid.get_pdfs())
        grid.step(1)
        ft1 = from_device(grid.get_pdfs())
        cells = rng.choice(np.flatnonzero(solid.reshape(-1) == 0), 200, replace=False)
        ids = ids_all[cells]
        assert rel_err(ft1[:, ids], _sample_update(ft, solid, cells, omega, g)) <= 1e-12, extra
        del ft, ft1
    m1 = from_device(grid.moments())
    assert abs(m1[0] - m0[0]) / m0[0] <= 1e-13


@pytest.fixture(scope="module")
def pack384():
    return lbm_inputs.sphere_pack(384, 8, 0.6, seed=4)[0]


@pytest.mark.parametrize("prec,sigma", [("f32", 1.0), ("f32s", 1.0), ("f16s", 1024.0)])
def test_384_precision_pack_sampled(prec, sigma, pack384):
    """The precision study's reduced storage forms on its 384^3 pack, indirect AA in the launch
    configuration the library picks by default (lattices in 1024-node blocks; neighbour ids by rank
    with FP32 and FP32-shifted storage, IDX with FP16-shifted).  Both AA kernels are sampled against the
    oracle's update under the same storage rounding, at the bars of the small-lattice precision tests,
    which hold while |f - w_i| < 2^-12 (checked on the state): FP32 relative 1e-6; FP32-shifted 2e-9
    in f; FP16-shifted 4 binary16 ulp of h, 4 * 2^-23 in f."""
    solid = pack384
    omega, g = 1.0, (1e-6, 0.0, 0.0)
    grid = make_grid(solid, "aa", addressing="indirect", precision=prec, omega=omega, g=g, f16_scale=sigma)
    assert grid.lattice_block == 1024
    assert grid.rank_lookup == (prec != "f16s")
    grid.cellmap = None
    grid._mask = None
    fl = solid.reshape(-1) == 0
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-4, seed=5))
    grid.init_equilibrium(to_device(np.ascontiguousarray(ru.reshape(4, -1)[:, fl])))
    del ru
    m0 = from_device(grid.moments())
    grid.step(3)
    _, w, _ = oracle.tables()
    rng = np.random.default_rng(3)
    ids_all = _fluid_ids(solid)
    kw = {"precision": prec, "sigma": sigma}
    for extra in (1, 2):
        ft = from_device(grid.get_pdfs())
        assert float(np.max(np.abs(ft - w[:, None]))) < 2.0 ** -12
        grid.step(1)
        ft1 = from_device(grid.get_pdfs())
        cells = rng.choice(np.flatnonzero(fl), 200, replace=False)
        ids = ids_all[cells]
        want = _sample_update(ft, solid, cells, omega, g, **kw)
        if prec == "f32":
            assert rel_err(ft1[:, ids], want) <= 1e-6, extra
        elif prec == "f32s":
            assert float(np.max(np.abs(ft1[:, ids] - want))) <= 2e-9, extra
        else:
            assert float(np.max(np.abs(ft1[:, ids] - want))) <= 4 * 2.0 ** -23, extra
        del ft, ft1
    m1 = from_device(grid.moments())
    assert abs(m1[0] - m0[0]) / m0[0] <= (1e-9 if prec == "f32s" else 1e-6)   # the small tests' mass bars
