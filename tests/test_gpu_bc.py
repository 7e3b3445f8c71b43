"""Open boundaries (velocity and pressure in-/outlets) on the GPU.

A duct with a velocity inlet, a pressure outlet, a moving lid, a resting
floor and spheres, run by every scheme (TS, OS push, OS pull, AA: both AA
parities, ET: its write side), both layouts, against the oracle's link
rules; the closed forms (uniform duct flow, Couette, pressure-driven
Poiseuille) on the GPU; canonical readout and upload through the rules; the
refusals (direct grids, bad arguments); open boundaries in batched
lattices (alone, mixed with walls-only lattices, graph and cooperative runs).
"""
import math

import numpy as np
import pytest
import torch

import lbm_inputs
import oracle
from lbm_cases import from_device, rel_err, to_device

pytestmark = pytest.mark.gpu

BC = {1: ("velocity", 1.0, (0.02, 0.0, 0.0)), 2: ("pressure", 0.995, (0.02, 0.0, 0.0)),
      3: ("velocity", 1.0, (0.01, 0.004, 0.0))}
C0 = np.array([0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0])


def duct(nx=20, ny=12, nz=10, seed=31):
    """uint8[nz, ny, nx]: floor z = 0 (wall), lid z = nz-1 (class 3), inlet x = 0
    (class 1), outlet x = nx-1 (class 2), plus a few resting spheres."""
    m = lbm_inputs.sphere_pack((nx, ny, nz), 2, 0.85, seed)[0].copy()
    m[:, :, 0] = 2
    m[:, :, nx - 1] = 3
    m[0] = 1
    m[nz - 1] = 4
    return m


def _grid(mask, scheme, layout="soa", precision="f64", omega=1.3, g=(0.0, 0.0, 0.0), f16_scale=1.0, bc=BC):
    import paper_1111_0922_amd as P
    nz, ny, nx = mask.shape
    grid = P.Grid(nx, ny, nz, addressing="indirect", layout=layout, precision=precision, omega=omega, g=g,
                  f16_scale=f16_scale, et_ghosts=(scheme == "et"))
    grid.build_idx(torch.from_numpy(np.ascontiguousarray(mask)).cuda())
    for cls, (kind, rho, u) in bc.items():
        grid.set_boundary(cls, kind, rho, u)
    grid.bind(scheme)
    return grid


def _state(mask, seed=32):
    ru = lbm_inputs.rho_u_field(mask.shape, lbm_inputs.velocity_noise(mask.shape, 1e-3, seed=seed))
    ru[1] += 0.02
    return oracle.init_equilibrium(ru, mask)


@pytest.mark.parametrize("layout", ["soa", "aos"])
@pytest.mark.parametrize("scheme", ["ts", "os_push", "os_pull", "aa", "et"])
@pytest.mark.parametrize("steps", [12, 13])
def test_open_boundaries_match_oracle(scheme, layout, steps):
    mask = duct()
    f0 = _state(mask)
    g = (1e-6, 0.0, 0.0)
    want = oracle.run_ts(f0, mask, steps, 1.3, g, bc=BC)
    grid = _grid(mask, scheme, layout, g=g)
    grid.set_pdfs(to_device(oracle.fluid_view(f0, mask)))
    grid.step(steps)
    assert rel_err(from_device(grid.get_pdfs()), oracle.fluid_view(want, mask)) <= 1e-12
    mo = oracle.moments(want, mask)
    m = from_device(grid.moments())
    assert abs(m[0] - mo[0]) / mo[0] <= 1e-13
    np.testing.assert_allclose(m[1:], mo[1:], rtol=1e-10, atol=1e-13 * mo[0])


@pytest.mark.parametrize("scheme", ["aa", "os_push", "et"])
def test_open_boundaries_trt_match_oracle(scheme):
    mask = duct(16, 9, 11, seed=33)
    f0 = _state(mask, 34)
    grid = _grid(mask, scheme)  # default Lambda = 3/16
    grid.set_pdfs(to_device(oracle.fluid_view(f0, mask)))
    grid.step(11, collider="trt")
    want = oracle.run_ts(f0, mask, 11, 1.3, (0, 0, 0), collider="trt",
                         omega_minus=oracle.trt_omega_minus(1.3, 3.0 / 16.0), bc=BC)
    assert rel_err(from_device(grid.get_pdfs()), oracle.fluid_view(want, mask)) <= 1e-12


@pytest.mark.parametrize("precision,bars", [("f32", (1e-6, 2e-5)), ("f32s", (1e-6, 2e-5))])
def test_open_boundaries_reduced_precision(precision, bars):
    mask = duct(16, 10, 9, seed=35)
    f0 = _state(mask, 36)
    q0 = oracle.quantize(f0, (mask != 0).astype(np.uint8), precision, 64.0)
    for steps, bar in zip((1, 20), bars):
        want = oracle.fluid_view(oracle.run_ts(q0, mask, steps, 1.3, (0, 0, 0), precision=precision, sigma=64.0,
                                               bc=BC), mask)
        grid = _grid(mask, "aa", precision=precision, f16_scale=64.0)
        grid.set_pdfs(to_device(oracle.fluid_view(q0, mask)))
        grid.step(steps)
        got = from_device(grid.get_pdfs())
        assert float(np.max(np.abs(got - want) / np.abs(want))) <= bar, steps


def test_open_boundaries_fp16_shifted():
    """FP16 shifted storage (sigma = 64) against the oracle with the same storage rounding.  The
    GPU collides in FP32 and the oracle in FP64, so a stored half can round the other way: one
    FP16 ulp of |v| < 1, divided by sigma, is 2^-10 / 64 in f; the bound allows one such flip
    per step."""
    mask = duct(16, 10, 9, seed=37)
    f0 = _state(mask, 38)
    sigma = 64.0
    q0 = oracle.quantize(f0, (mask != 0).astype(np.uint8), "f16s", sigma)
    for steps in (1, 5):
        want = oracle.fluid_view(oracle.run_ts(q0, mask, steps, 1.3, (0, 0, 0), precision="f16s", sigma=sigma,
                                               bc=BC), mask)
        grid = _grid(mask, "aa", precision="f16s", f16_scale=sigma)
        grid.set_pdfs(to_device(oracle.fluid_view(q0, mask)))
        grid.step(steps)
        got = from_device(grid.get_pdfs())
        assert float(np.max(np.abs(got - want))) <= steps * 2.0 ** -10 / sigma, steps


@pytest.mark.parametrize("scheme", ["aa", "os_pull"])
def test_readout_and_upload_through_the_rules(scheme):
    """At odd t (AA) and always (OS pull) the canonical state passes the rules:
    upload then readout returns the state up to one rounding at boundary links."""
    mask = duct()
    f0 = _state(mask)
    grid = _grid(mask, scheme)
    grid.set_pdfs(to_device(oracle.fluid_view(f0, mask)))
    grid.step(3)
    f3 = from_device(grid.get_pdfs())
    grid.set_pdfs(to_device(f3))
    assert rel_err(from_device(grid.get_pdfs()), f3) <= 1e-15
    # init_equilibrium through the rules: the readout is the equilibrium
    grid.init_equilibrium()
    fe = from_device(grid.get_pdfs())
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    assert float(np.max(np.abs(fe - w[:, None]))) <= 1e-16


def test_uniform_duct_flow_is_fixed_on_gpu():
    nx, ny, nz = 24, 8, 6
    U = (0.02, -0.004, 0.003)
    m = np.zeros((nz, ny, nx), np.uint8)
    m[:, :, 0] = 2
    m[:, :, nx - 1] = 3
    ru = lbm_inputs.rho_u_field(m.shape)
    ru[1:] = np.array(U)[:, None, None, None]
    f0 = oracle.fluid_view(oracle.init_equilibrium(ru, m), m)
    bc = {1: ("velocity", 1.0, U), 2: ("pressure", 1.0, U)}
    for scheme in ("aa", "ts", "os_push", "os_pull", "et"):
        grid = _grid(m, scheme, bc=bc)
        grid.set_pdfs(to_device(f0))
        grid.step(40, collider="trt")
        assert float(np.max(np.abs(from_device(grid.get_pdfs()) - f0))) <= 1e-15, scheme


@pytest.mark.parametrize("omega", [0.8, 1.6])
def test_couette_is_linear_on_gpu(omega):
    nz, Uw = 18, 0.01
    H = nz - 2
    nu = (1.0 / omega - 0.5) / 3.0
    m = np.zeros((nz, 2, 2), np.uint8)
    m[0] = 1
    m[nz - 1] = 2
    grid = _grid(m, "aa", omega=omega, bc={1: ("velocity", 1.0, (Uw, 0, 0))})
    grid.init_equilibrium()
    m0 = from_device(grid.moments())[0]
    grid.step(int(6 * H * H / nu) // 2 * 2)
    f = from_device(grid.get_pdfs()).reshape(19, H, 2, 2)
    ux = np.tensordot(C0, f, axes=(0, 0)) / f.sum(axis=0)
    z = np.arange(1, nz - 1)[:, None, None]
    assert np.abs(ux - Uw * (z - 0.5) / H).max() / Uw < 1e-10
    assert abs(from_device(grid.moments())[0] - m0) / m0 < 1e-11


def test_pressure_driven_slit_on_gpu():
    nx, nz = 42, 10
    H, L = nz - 2, nx - 2
    omega = 1.0 / (0.5 + math.sqrt(3.0) / 4.0)
    nu = (1.0 / omega - 0.5) / 3.0
    drho = 1e-5
    m = np.zeros((nz, 1, nx), np.uint8)
    m[0] = 1
    m[nz - 1] = 1
    m[1:-1, :, 0] = 2
    m[1:-1, :, nx - 1] = 3
    grid = _grid(m, "aa", omega=omega,
                 bc={1: ("pressure", 1 + drho / 2, (0, 0, 0)), 2: ("pressure", 1 - drho / 2, (0, 0, 0))})
    grid.init_equilibrium()
    grid.step((int(6 * H * H / nu) + 8 * L * L) // 2 * 2)
    f = from_device(grid.get_pdfs()).reshape(19, H, L)   # fluid nodes: z = 1..H, x = 1..L
    rho = f.sum(axis=0)
    ux = np.tensordot(C0, f, axes=(0, 0)) / rho
    rm = rho.mean(axis=0)
    x1, x2 = L // 4, 3 * L // 4
    g = (rm[x1] - rm[x2]) / (x2 - x1) / 3.0
    z = np.arange(1, nz - 1)
    exact = g / (2 * nu) * (z - 0.5) * (H + 0.5 - z)
    assert np.abs(ux[:, L // 2] - exact).max() / exact.max() < 1e-4


def test_refusals():
    import paper_1111_0922_amd as P
    mask = duct()
    aa = _grid(mask, "aa", precision="f32")
    aa.init_equilibrium()
    direct = P.Grid(8, 8, 8, wall_z=True)
    with pytest.raises(P.LbmError):
        direct.set_boundary(1, "velocity", 1.0, (0.01, 0, 0))
    with pytest.raises(P.LbmError):
        aa.set_boundary(5, "velocity", 1.0, (0.01, 0, 0))
    with pytest.raises(P.LbmError):
        aa.set_boundary(1, "pressure", -1.0, (0, 0, 0))


def _batch_lattices(precision):
    """Two open-boundary ducts (one started at odd parity, other classes and sizes) and a
    walls-only porous lattice: (grid, steps before the batch) pairs, built the same way each call."""
    import paper_1111_0922_amd as P
    out = []
    for k, (shape, seed, bc, pre) in enumerate([((20, 12, 10), 31, BC, 0), ((16, 9, 11), 33, {1: ("pressure", 1.004, (0, 0, 0)),
                                                2: ("pressure", 0.996, (0, 0, 0)), 3: ("velocity", 1.0, (0, 0.01, 0))}, 1),
                                               ((18, 14, 12), 35, {}, 0)]):
        mask = duct(*shape, seed=seed) if bc else lbm_inputs.sphere_pack(shape, 3, 0.6, seed)[0]
        grid = _grid(mask, "aa", precision=precision, f16_scale=64.0, bc=bc)
        grid.set_pdfs(to_device(oracle.fluid_view(_state(mask, seed + 1), mask)))
        if pre:
            grid.step(pre)
        out.append(grid)
    return out


@pytest.mark.parametrize("precision", ["f64", "f32", "f32s", "f16s"])
@pytest.mark.parametrize("mode", ["graph", "cooperative"])
def test_batched_open_boundaries_equal_alone(precision, mode):
    """Open-boundary lattices in a batch (mixed with a walls-only one) evolve to the bits of
    the same lattices stepped alone, states and moments, over two runs."""
    import paper_1111_0922_amd as P
    K = 7
    alone = []
    for grid in _batch_lattices(precision):
        grid.step(2 * K)
        alone.append((from_device(grid.get_pdfs()), from_device(grid.moments())))
    batch = P.Batch(4, 1024, precision, mode=mode)
    grids = [(batch.add(g), g) for g in _batch_lattices(precision)]
    for _ in range(2):
        m = batch.run(K)
    for (slot, grid), (f_alone, m_alone) in zip(grids, alone):
        assert np.array_equal(from_device(grid.get_pdfs()).view(np.int64), f_alone.view(np.int64)), slot
        assert np.array_equal(m[slot].view(np.int64), m_alone.view(np.int64)), slot


def test_batched_open_boundaries_match_oracle():
    """FP64 duct in a batch against the oracle's link rules."""
    import paper_1111_0922_amd as P
    mask = duct()
    f0 = _state(mask)
    grid = _grid(mask, "aa")
    grid.set_pdfs(to_device(oracle.fluid_view(f0, mask)))
    batch = P.Batch(2, 256, "f64")
    s = batch.add(grid)
    m = batch.run(13)
    want = oracle.run_ts(f0, mask, 13, 1.3, (0.0, 0.0, 0.0), bc=BC)
    assert rel_err(from_device(grid.get_pdfs()), oracle.fluid_view(want, mask)) <= 1e-12
    mo = oracle.moments(want, mask)
    assert abs(m[s][0] - mo[0]) / mo[0] <= 1e-13
    np.testing.assert_allclose(m[s][1:], mo[1:], rtol=1e-10, atol=1e-13 * mo[0])
