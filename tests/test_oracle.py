"""Pins of the FP64 oracle against facts fixed outside it.

Each test checks the oracle against mathematics or hand-worked values, never
against a retyped copy of its own formulas:
  * lattice tables  -- golden ordering file and the isotropy identities of D3Q19;
  * equilibrium     -- its velocity moments up to second order;
  * Guo forcing     -- its moments (zero mass, (1-w/2)F momentum, stress term);
  * collision       -- exact mass conservation and momentum gain F per node;
                       TRT: equal rates reduce to BGK, even and odd
                       non-equilibrium parts decay by (1 - w+) and (1 - w-);
  * propagation     -- an exact permutation, built here with numpy rolls;
  * whole runs      -- mass conservation, momentum growth M g per step,
                       the rest state, Poiseuille flow (closed form, exact at
                       the TRT 'magic' relaxation), shear-wave viscosity and the
                       slit permeability;
  * IDX             -- a hand-worked 4^3 example and the link symmetry;
  * open boundaries -- uniform flow through a velocity inlet and a pressure
                       outlet is fixed, Couette flow is exactly linear, a
                       pressure box takes its density, pressure-driven slit
                       flow is Poiseuille flow, resting wall classes are plain
                       bounce-back;
  * binary16 rounding -- numpy's float16 conversion.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import lbm_inputs
import oracle
from golden_io import d3q19_ordering, idx_4cube

C, W, OPP = d3q19_ordering()
Wf = np.array([float(w) for w in W])
G = (1e-6, 0.0, 0.0)


# ---------------------------------------------------------------- tables
def test_tables_match_golden_ordering():
    c, w, opp = oracle.tables()
    np.testing.assert_array_equal(c, C)
    np.testing.assert_array_equal(opp, OPP)
    np.testing.assert_allclose(w, Wf, rtol=0, atol=1e-17)


def test_lattice_isotropy():
    """sum w = 1, sum w c_a c_b = d_ab/3, 4th moment = (d d + d d + d d)/9 (exact, in fractions)."""
    c, _, opp = oracle.tables()
    assert len({tuple(v) for v in c}) == 19
    assert sum(W) == 1
    for a in range(3):
        for b in range(3):
            assert sum(W[i] * int(C[i, a] * C[i, b]) for i in range(19)) == (Fraction(1, 3) if a == b else 0)
            for g in range(3):
                assert sum(W[i] * int(C[i, a] * C[i, b] * C[i, g]) for i in range(19)) == 0
                for d in range(3):
                    m4 = sum(W[i] * int(C[i, a] * C[i, b] * C[i, g] * C[i, d]) for i in range(19))
                    want = ((a == b) * (g == d) + (a == g) * (b == d) + (a == d) * (b == g))
                    assert m4 * 9 == want
    for i in range(19):
        np.testing.assert_array_equal(c[opp[i]], -c[i])


# ---------------------------------------------------------------- equilibrium / forcing / collision
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_equilibrium_moments(seed):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.1 * rng.standard_normal()
    u = 0.05 * rng.standard_normal(3)
    feq = oracle.equilibrium(rho, u)
    assert abs(feq.sum() - rho) < 1e-15
    np.testing.assert_allclose(C.T @ feq, rho * u, rtol=0, atol=1e-16)
    P = np.einsum("ia,ib,i->ab", C, C, feq)
    np.testing.assert_allclose(P, rho * np.outer(u, u) + rho / 3.0 * np.eye(3), rtol=0, atol=1e-15)


@pytest.mark.parametrize("omega", [0.7, 1.0, 1.6])
def test_guo_source_moments(omega):
    rng = np.random.default_rng(7)
    rho = 1.02
    u = 0.03 * rng.standard_normal(3)
    g = 1e-3 * rng.standard_normal(3)
    F = rho * g
    S = oracle.guo_source(rho, u, omega, g)
    k = 1.0 - 0.5 * omega
    assert abs(S.sum()) < 1e-18
    np.testing.assert_allclose(C.T @ S, k * F, rtol=1e-13, atol=1e-19)
    P = np.einsum("ia,ib,i->ab", C, C, S)
    np.testing.assert_allclose(P, k * (np.outer(u, F) + np.outer(F, u)), rtol=1e-12, atol=1e-19)


@pytest.mark.parametrize("omega", [0.6, 1.0, 1.9])
def test_collision_conserves_mass_and_adds_force(omega):
    rng = np.random.default_rng(3)
    f = Wf * (1.0 + 0.01 * rng.standard_normal(19))
    g = np.array([1e-4, -2e-4, 3e-5])
    fs = oracle.collide_node(f, omega, g)
    rho = f.sum()
    assert abs(fs.sum() - rho) <= 4 * np.finfo(float).eps * rho
    # with u = (j + rho g/2)/rho the post-collision momentum is j + rho g exactly
    np.testing.assert_allclose(C.T @ fs, C.T @ f + rho * g, rtol=0, atol=4e-16)


def test_collision_at_omega_one_is_equilibrium_plus_source():
    rng = np.random.default_rng(4)
    f = Wf * (1.0 + 0.01 * rng.standard_normal(19))
    fs = oracle.collide_node(f, 1.0, (0, 0, 0))
    rho = f.sum()
    u = (C.T @ f) / rho
    np.testing.assert_allclose(fs, oracle.equilibrium(rho, u), rtol=0, atol=1e-17)


def test_identity_collider_is_identity():
    f = np.random.default_rng(5).standard_normal(19)
    np.testing.assert_array_equal(oracle.collide_node(f, 1.3, G, "identity"), f)


def _odd_even_perturbation(seed):
    """A zero-mass, zero-momentum perturbation split into its even and odd parts."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(19) * 1e-3
    # project out mass and momentum (weighted least squares onto 1, c_x, c_y, c_z)
    B = np.column_stack([np.ones(19), C])
    d -= B @ np.linalg.lstsq(B, d, rcond=None)[0]
    opp = np.array([0] + [i + 1 if i % 2 else i - 1 for i in range(1, 19)])
    return 0.5 * (d + d[opp]), 0.5 * (d - d[opp])


@pytest.mark.parametrize("omega", [0.7, 1.0, 1.7])
def test_trt_equal_rates_is_bgk(omega):
    rng = np.random.default_rng(31)
    f = Wf * (1.0 + 0.01 * rng.standard_normal(19))
    g = np.array([2e-4, -1e-4, 5e-5])
    np.testing.assert_allclose(oracle.collide_node(f, omega, g, "trt", omega_minus=omega),
                               oracle.collide_node(f, omega, g), rtol=0, atol=4e-17)


@pytest.mark.parametrize("wp,wm", [(1.2, 0.4), (0.8, 1.9), (1.5, 1.5)])
def test_trt_even_and_odd_parts_relax_at_their_rates(wp, wm):
    """At equilibrium plus a mass- and momentum-free perturbation, rho and u do not
    move, so the even part of the perturbation leaves scaled by 1 - w+ and the odd
    part by 1 - w-; mass and momentum (+ rho g) stay exact."""
    rho, u = 1.03, np.array([0.02, -0.01, 0.015])
    feq = oracle.equilibrium(rho, u)
    de, do = _odd_even_perturbation(7)
    out = oracle.collide_node(feq + de + do, wp, (0, 0, 0), "trt", omega_minus=wm)
    np.testing.assert_allclose(out, feq + (1 - wp) * de + (1 - wm) * do, rtol=0, atol=6e-17)
    g = np.array([1e-4, 3e-5, -2e-4])
    f = feq + de + do
    fs = oracle.collide_node(f, wp, g, "trt", omega_minus=wm)
    assert abs(fs.sum() - f.sum()) <= 4 * np.finfo(float).eps * rho
    np.testing.assert_allclose(C.T @ fs, C.T @ f + f.sum() * g, rtol=0, atol=4e-16)


# ---------------------------------------------------------------- propagation = permutation
def _numpy_pull_permutation(B, solid):
    """A[i][x] = B[i][x - c_i], or B[opp i][x] when x - c_i is solid (periodic box)."""
    A = np.zeros_like(B)
    for i in range(19):
        shift = (int(C[i, 2]), int(C[i, 1]), int(C[i, 0]))  # array axes are z, y, x
        src = np.roll(B[i], shift, axis=(0, 1, 2))
        src_solid = np.roll(solid, shift, axis=(0, 1, 2)).astype(bool)
        A[i] = np.where(src_solid, B[OPP[i]], src)
    A[:, solid.astype(bool)] = 0.0
    return A


@pytest.mark.parametrize("shape", [(5, 6, 7), (8, 4, 3), (1, 1, 9)])
def test_stream_only_step_is_exact_permutation(shape):
    rng = np.random.default_rng(11)
    solid = (rng.random(shape) < 0.25).astype(np.uint8)
    # random 64-bit patterns, NaN payloads included: only a permutation keeps them
    bits = rng.integers(0, 2**63, size=(19,) + shape, dtype=np.int64)
    f = bits.view(np.float64).copy()
    f[:, solid.astype(bool)] = 0.0
    got = oracle.run_ts(f, solid, 1, 1.3, G, collider="identity")
    want = _numpy_pull_permutation(f, solid)
    np.testing.assert_array_equal(got.view(np.int64), want.view(np.int64))


def test_stream_only_two_steps_compose():
    rng = np.random.default_rng(12)
    shape = (6, 5, 4)
    solid = (rng.random(shape) < 0.3).astype(np.uint8)
    f = rng.standard_normal((19,) + shape)
    f[:, solid.astype(bool)] = 0.0
    got = oracle.run_ts(f, solid, 2, 1.0, G, collider="identity")
    want = _numpy_pull_permutation(_numpy_pull_permutation(f, solid), solid)
    np.testing.assert_array_equal(got, want)


def test_non_periodic_axis_bounces_back():
    """Outside a non-periodic axis behaves like a solid cell: same as an explicit wall layer."""
    rng = np.random.default_rng(13)
    inner = (4, 3, 5)
    f_in = rng.standard_normal((19,) + inner)
    got = oracle.run_ts(f_in, np.zeros(inner, np.uint8), 1, 1.0, G, periodic=(1, 1, 0), collider="identity")
    padded = np.zeros((19, inner[0] + 2) + inner[1:])
    padded[:, 1:-1] = f_in
    solid = np.zeros((inner[0] + 2,) + inner[1:], np.uint8)
    solid[0] = solid[-1] = 1
    want = oracle.run_ts(padded, solid, 1, 1.0, G, periodic=(1, 1, 1), collider="identity")[:, 1:-1]
    np.testing.assert_array_equal(got, want)


# ---------------------------------------------------------------- whole runs
def _config1_state():
    solid = lbm_inputs.channel_mask(32, 32, 32)
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=1))
    return solid, oracle.init_equilibrium(ru, solid)


def test_mass_conservation_config1():
    solid, f0 = _config1_state()
    f = oracle.run_ts(f0, solid, 100, 1.0, G)
    M0 = oracle.moments(f0, solid)[0]
    M1 = oracle.moments(f, solid)[0]
    assert abs(M1 - M0) / M0 <= 1e-13


def test_mass_conservation_porous():
    solid, _ = lbm_inputs.sphere_pack(24, 3, 0.5, seed=9)
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=2))
    f0 = oracle.init_equilibrium(ru, solid)
    f = oracle.run_ts(f0, solid, 100, 1.6, G)
    M0, M1 = oracle.moments(f0, solid)[0], oracle.moments(f, solid)[0]
    assert abs(M1 - M0) / M0 <= 1e-13


def test_momentum_grows_by_Mg_per_step_in_periodic_box():
    shape = (8, 8, 8)
    solid = np.zeros(shape, np.uint8)
    ru = lbm_inputs.rho_u_field(shape, lbm_inputs.velocity_noise(shape, 1e-3, seed=3))
    f0 = oracle.init_equilibrium(ru, solid)
    g = (1e-5, -2e-5, 3e-6)
    f = oracle.run_ts(f0, solid, 50, 1.3, g)
    m0, m1 = oracle.moments(f0, solid), oracle.moments(f, solid)
    want = m0[1:] + 50 * m0[0] * np.array(g)
    np.testing.assert_allclose(m1[1:], want, rtol=1e-11, atol=0)


def test_rest_state_is_fixed_point():
    shape = (4, 5, 6)
    solid = np.zeros(shape, np.uint8)
    solid[1, 2, 3] = 1
    f0 = oracle.init_equilibrium(lbm_inputs.rho_u_field(shape), solid)
    f = oracle.run_ts(f0, solid, 10, 1.4, (0, 0, 0))
    np.testing.assert_allclose(f, f0, rtol=0, atol=2e-16)


def _poiseuille(omega, nz=32, steps=None, omega_minus=None):
    solid = lbm_inputs.channel_mask(2, 2, nz)
    nu = (1.0 / omega - 0.5) / 3.0
    H = nz - 2
    steps = steps or int(5 * H * H / nu)
    f = oracle.init_equilibrium(lbm_inputs.rho_u_field(solid.shape), solid)
    collider = "bgk" if omega_minus is None else "trt"
    f = oracle.run_ts(f, solid, steps, omega, G, collider=collider, omega_minus=omega_minus)
    _, u = oracle.macroscopic(f, solid, G)
    ux = u[0, 1:-1, 0, 0]
    z = np.arange(1, nz - 1, dtype=np.float64)
    exact = G[0] / (2 * nu) * (z - 0.5) * (H + 0.5 - z)  # walls half-way, at z = 1/2 and H + 1/2
    return f, solid, ux, exact, nu


def test_poiseuille_curvature_and_profile():
    _, _, ux, exact, nu = _poiseuille(1.0)
    curv = ux[2:] - 2 * ux[1:-1] + ux[:-2]
    np.testing.assert_allclose(curv, -G[0] / nu, rtol=1e-9)
    assert np.abs(ux - exact).max() / exact.max() < 1e-3


def test_poiseuille_slip_follows_magic_parameter():
    """BGK is TRT with Lambda = (1/omega - 1/2)^2: the bounce-back slip is (g/nu)(16 Lambda - 3)/24."""
    for omega in (1.0, 0.8):
        _, _, ux, exact, nu = _poiseuille(omega)
        lam = (1.0 / omega - 0.5) ** 2
        slip = (ux - exact).mean()
        assert abs(slip / (G[0] / nu * (16 * lam - 3) / 24) - 1) < 5e-3


def test_poiseuille_exact_at_magic_relaxation():
    omega = 1.0 / (0.5 + math.sqrt(3.0) / 4.0)  # Lambda = 3/16
    _, _, ux, exact, _ = _poiseuille(omega)
    assert np.abs(ux - exact).max() / exact.max() < 1e-9


@pytest.mark.parametrize("omega", [0.8, 1.0, 1.6])
def test_trt_poiseuille_exact_at_lambda_3_16(omega):
    """With TRT the bounce-back wall position depends only on Lambda: at
    Lambda = 3/16 the half-way parabola is exact for any w+."""
    wm = oracle.trt_omega_minus(omega, 3.0 / 16.0)
    _, _, ux, exact, _ = _poiseuille(omega, omega_minus=wm)
    assert np.abs(ux - exact).max() / exact.max() < 1e-9


def test_trt_poiseuille_slip_follows_lambda():
    """Away from 3/16 the slip is (g/nu)(16 Lambda - 3)/24, set by w- at fixed w+."""
    omega = 1.0
    for lam in (0.05, 0.5):
        _, _, ux, exact, nu = _poiseuille(omega, omega_minus=oracle.trt_omega_minus(omega, lam))
        slip = (ux - exact).mean()
        assert abs(slip / (G[0] / nu * (16 * lam - 3) / 24) - 1) < 5e-3


def test_slit_permeability_closed_form():
    """Darcy k of a slit of width H in a box of height nz: H^3/(12 nz) (1 + 1/(2 H^2))."""
    omega = 1.0 / (0.5 + math.sqrt(3.0) / 4.0)
    f, solid, _, _, _ = _poiseuille(omega)
    nz = solid.shape[0]
    H = nz - 2
    phi = float((solid == 0).mean())
    k = oracle.permeability(oracle.moments(f, solid), G, omega, phi)
    want = H ** 3 / (12.0 * nz) * (1 + 1.0 / (2 * H * H))
    assert abs(k / want - 1) < 1e-9


@pytest.mark.parametrize("omega,tol,omega_minus", [(1.0, 1e-5, None), (1.6, 3e-3, None), (1.0, 3e-3, 1.6),
                                                   (1.0, 5e-3, 0.5)])
def test_shear_wave_viscosity(omega, tol, omega_minus):
    """Decay rate nu k^2 (up to O(k^2) relative terms) with nu = (1/w - 1/2)/3;
    under TRT only w+ sets nu (w- would change it four-fold here)."""
    L = 64
    solid = np.zeros((L, 1, 1), np.uint8)
    z = np.arange(L)
    ru = lbm_inputs.rho_u_field(solid.shape)
    ru[1, :, 0, 0] = 1e-4 * np.sin(2 * np.pi * z / L)
    f = oracle.init_equilibrium(ru, solid)
    k = 2 * np.pi / L

    def amp(f):
        _, u = oracle.macroscopic(f, solid, (0, 0, 0))
        return (u[0, :, 0, 0] * np.sin(k * z)).sum() * 2 / L

    kw = dict(collider="bgk" if omega_minus is None else "trt", omega_minus=omega_minus)
    f = oracle.run_ts(f, solid, 200, omega, (0, 0, 0), **kw)
    a1 = amp(f)
    f = oracle.run_ts(f, solid, 2000, omega, (0, 0, 0), **kw)
    a2 = amp(f)
    nu = (1.0 / omega - 0.5) / 3.0
    assert abs(-math.log(a2 / a1) / (k * k * 2000) / nu - 1) < tol


# ---------------------------------------------------------------- IDX
def test_idx_hand_worked_4cube():
    solid_cells, nodes = idx_4cube()
    solid = np.zeros((4, 4, 4), np.uint8)
    for c in solid_cells:
        solid.reshape(-1)[c] = 1
    cellmap, idx, nf = oracle.build_idx(solid)
    assert nf == 62
    for n, want in nodes.items():
        assert list(idx[:, n]) == want


def test_idx_link_symmetry_and_counts():
    solid, _ = lbm_inputs.sphere_pack((10, 9, 8), 2, 0.55, seed=21)
    cellmap, idx, nf = oracle.build_idx(solid)
    assert nf == int((solid == 0).sum())
    flat = cellmap.reshape(-1)
    assert (flat[solid.reshape(-1) == 1] == -1).all()
    np.testing.assert_array_equal(flat[solid.reshape(-1) == 0], np.arange(nf))
    for k in range(18):
        kk = OPP[k + 1] - 1
        m = idx[k]
        ok = m >= 0
        np.testing.assert_array_equal(idx[kk, m[ok]], np.arange(nf)[ok])
    # number of fluid->solid links equals the count of solid neighbours, direction by direction
    for k in range(18):
        shift = tuple(-int(v) for v in C[k + 1][::-1])
        nb_solid = np.roll(solid, shift, axis=(0, 1, 2)).reshape(-1)[solid.reshape(-1) == 0]
        assert int((idx[k] == -1).sum()) == int(nb_solid.sum())


# ---------------------------------------------------------------- storage rounding
def test_round_half_matches_ieee_binary16():
    rng = np.random.default_rng(17)
    v = np.concatenate([
        rng.standard_normal(20000) * 10.0 ** rng.integers(-9, 5, 20000),
        np.array([65504.0, 65519.99, 65520.0, 7e4, 2.0 ** -24, 2.0 ** -25, 1.5 * 2.0 ** -25, 2.0 ** -14,
                  1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11, -3.0e-6, 0.0]),
    ])
    got = oracle.round_half(v)
    want = v.astype(np.float16).astype(np.float64)
    np.testing.assert_array_equal(got, want)


def test_quantize_forms():
    rng = np.random.default_rng(18)
    solid = np.zeros((3, 3, 3), np.uint8)
    f = Wf[:, None, None, None] * (1 + 1e-3 * rng.standard_normal((19, 3, 3, 3)))
    np.testing.assert_array_equal(oracle.quantize(f, solid, "f32"), f.astype(np.float32).astype(np.float64))
    sigma = 1024.0
    q32 = oracle.quantize(f, solid, "f32s", sigma)
    d = ((f - Wf[:, None, None, None]) * sigma).astype(np.float32).astype(np.float64)
    np.testing.assert_array_equal(q32, Wf[:, None, None, None] + d / sigma)
    q = oracle.quantize(f, solid, "f16s", sigma)
    h = ((f - Wf[:, None, None, None]) * sigma).astype(np.float16).astype(np.float64)
    np.testing.assert_array_equal(q, Wf[:, None, None, None] + h / sigma)


def test_brick_ordering_is_a_renumbering():
    """Brick-ordered ids number the same fluid cells; links map onto each other under the renumbering."""
    solid, _ = lbm_inputs.sphere_pack((10, 9, 7), 2, 0.5, seed=1)
    cm0, idx0, nf = oracle.build_idx(solid)
    cm1, idx1, nf1 = oracle.build_idx(solid, brick=(4, 3, 2))
    assert nf1 == nf
    assert np.array_equal(cm0 >= 0, cm1 >= 0)
    # id of brick (0,0,0)'s first fluid cell is 0; cells of brick (0,0,0) come first
    first = cm1[:2, :3, :4]
    assert sorted(first[first >= 0].ravel().tolist()) == list(range(int((first >= 0).sum())))
    # renumbering map new -> old
    new_to_old = np.empty(nf, np.int64)
    new_to_old[cm1[cm1 >= 0]] = cm0[cm1 >= 0]
    old_to_new = np.empty(nf, np.int64)
    old_to_new[new_to_old] = np.arange(nf)
    mapped = np.where(idx0 >= 0, old_to_new[np.maximum(idx0, 0)], -1)
    np.testing.assert_array_equal(idx1[:, old_to_new], mapped)
    # a brick covering the box is the lexicographic order
    cm2, idx2, _ = oracle.build_idx(solid, brick=(10, 9, 7))
    np.testing.assert_array_equal(cm2, cm0)


# ---------------------------------------------------------------- open boundaries
def test_bc_uniform_flow_through_velocity_inlet_and_pressure_outlet_is_fixed():
    """f = f^eq(1, U) everywhere is the steady state of a duct between a
    velocity inlet (U) and a pressure outlet (rho 1, U): both link rules give
    back exactly the equilibrium populations."""
    nx, ny, nz = 10, 3, 4
    U = (0.02, -0.004, 0.003)
    m = np.zeros((nz, ny, nx), np.uint8)
    m[:, :, 0] = 2
    m[:, :, nx - 1] = 3
    ru = lbm_inputs.rho_u_field(m.shape)
    ru[1:] = np.array(U)[:, None, None, None]
    f0 = oracle.init_equilibrium(ru, m)
    bc = {1: ("velocity", 1.0, U), 2: ("pressure", 1.0, U)}
    for collider, wm in (("bgk", None), ("trt", 0.7)):
        f = oracle.run_ts(f0, m, 40, 1.3, (0, 0, 0), collider=collider, omega_minus=wm, bc=bc)
        np.testing.assert_allclose(f, f0, rtol=0, atol=1e-15)  # f >= 0.02: a few ulp


@pytest.mark.parametrize("omega", [0.8, 1.0, 1.6])
def test_bc_couette_profile_is_linear_and_mass_conserved(omega):
    """A lid moving tangentially at U over a fixed wall: the steady profile is
    the straight line u = U (z - 1/2)/H between the half-way walls, which
    bounce-back reproduces exactly, and the moving wall adds no mass."""
    nz, Uw = 18, 0.01
    H = nz - 2
    nu = (1.0 / omega - 0.5) / 3.0
    m = np.zeros((nz, 2, 2), np.uint8)
    m[0] = 1
    m[nz - 1] = 2
    f = oracle.init_equilibrium(lbm_inputs.rho_u_field(m.shape), m)
    M0 = oracle.moments(f, m)[0]
    f = oracle.run_ts(f, m, int(6 * H * H / nu), omega, (0, 0, 0), bc={1: ("velocity", 1.0, (Uw, 0, 0))})
    _, u = oracle.macroscopic(f, m, (0, 0, 0))
    z = np.arange(1, nz - 1)
    assert np.abs(u[0, 1:-1] - (Uw * (z - 0.5) / H)[:, None, None]).max() / Uw < 1e-10
    assert abs(oracle.moments(f, m)[0] - M0) / M0 < 1e-11


def test_bc_pressure_boundary_sets_the_density():
    """A box enclosed by pressure cells of density 1.02 (u = 0) relaxes from
    rest at rho = 1 to rho = 1.02; f^eq(1.02, 0) is an exact fixed point."""
    nx, ny, nz = 7, 6, 5
    m = np.full((nz, ny, nx), 2, np.uint8)
    m[1:-1, 1:-1, 1:-1] = 0
    bc = {1: ("pressure", 1.02, (0, 0, 0))}
    f = oracle.init_equilibrium(lbm_inputs.rho_u_field(m.shape), m)
    f = oracle.run_ts(f, m, 300, 1.0, (0, 0, 0), bc=bc)
    rho, _ = oracle.macroscopic(f, m, (0, 0, 0))
    assert np.abs(rho[m == 0] - 1.02).max() < 1e-14
    ru = lbm_inputs.rho_u_field(m.shape)
    ru[0] = 1.02
    feq = oracle.init_equilibrium(ru, m)
    np.testing.assert_allclose(oracle.run_ts(feq, m, 7, 1.4, (0, 0, 0), bc=bc), feq, rtol=0, atol=1e-15)


def test_bc_pressure_driven_slit_is_poiseuille():
    """Two pressure boundaries drive a slit flow: where it is developed, the
    profile is the body-force Poiseuille parabola for the measured density
    gradient, g = c_s^2 d(rho)/dx, up to the compressibility O(d rho)."""
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
    f = oracle.init_equilibrium(lbm_inputs.rho_u_field(m.shape), m)
    bc = {1: ("pressure", 1 + drho / 2, (0, 0, 0)), 2: ("pressure", 1 - drho / 2, (0, 0, 0))}
    f = oracle.run_ts(f, m, int(6 * H * H / nu) + 8 * L * L, omega, (0, 0, 0), bc=bc)
    rho, u = oracle.macroscopic(f, m, (0, 0, 0))
    rm = rho[1:-1, 0, :].mean(axis=0)
    x1, x2 = nx // 4, 3 * nx // 4
    g = (rm[x1] - rm[x2]) / (x2 - x1) / 3.0
    z = np.arange(1, nz - 1)
    exact = g / (2 * nu) * (z - 0.5) * (H + 0.5 - z)
    assert np.abs(u[0, 1:-1, 0, nx // 2] - exact).max() / exact.max() < 1e-4
    assert rm[1] > rm[x1] > rm[x2] > rm[-2]


def test_bc_still_wall_classes_are_plain_bounce_back():
    solid = lbm_inputs.sphere_pack((12, 10, 9), 3, 0.6, seed=5)[0]
    m = solid.copy()
    m[solid == 1] = 2 + (np.arange(int(solid.sum())) % 3).astype(np.uint8)  # classes 1..3
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=3))
    f0 = oracle.init_equilibrium(ru, solid)
    want = oracle.run_ts(f0, solid, 9, 1.4, (1e-5, 0, 0))
    bc = {1: ("wall", 1.0, (0.1, 0, 0)), 2: ("velocity", 1.0, (0, 0, 0)), 3: ("velocity", 1.3, (0, 0, 0))}
    got = oracle.run_ts(f0, m, 9, 1.4, (1e-5, 0, 0), bc=bc)
    assert np.array_equal(got, want)


def test_bc_idx_codes():
    """IDX holds -m for a neighbour cell of mask value m (-1 for plain solid)."""
    m = np.zeros((4, 4, 4), np.uint8)
    m[0, 0, 0] = 1
    m[2, 1, 3] = 4
    cellmap, idx, _ = oracle.build_idx(m)
    # the fluid cell at (x, y, z) = (2, 1, 2) has the value-4 cell at +x (direction 1, row 0)
    assert idx[0][cellmap[2, 1, 2]] == -4
    # the fluid cell at (0, 0, 1) has the plain solid cell at -z (direction 6, row 5)
    assert idx[5][cellmap[1, 0, 0]] == -1
    assert sorted(set(idx[idx < 0].tolist())) == [-4, -1]


def test_mask_values_above_five_are_plain_walls():
    """Mask values 2..5 name boundary classes 1..4; every other non-zero value is a plain wall:
    -1 in IDX and plain bounce-back, even when every class is an open boundary."""
    solid = lbm_inputs.sphere_pack((12, 10, 9), 3, 0.6, seed=8)[0]
    m = solid.copy()
    big = np.array([6, 7, 9, 64, 200, 255], np.uint8)
    m[solid == 1] = big[np.arange(int(solid.sum())) % len(big)]
    c1, idx1, nf1 = oracle.build_idx(solid)
    c2, idx2, nf2 = oracle.build_idx(m)
    assert nf1 == nf2
    np.testing.assert_array_equal(c1, c2)
    np.testing.assert_array_equal(idx1, idx2)
    assert set(np.unique(idx2[idx2 < 0]).tolist()) == {-1}
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=4))
    f0 = oracle.init_equilibrium(ru, solid)
    bc = {1: ("velocity", 1.0, (0.05, 0, 0)), 2: ("pressure", 1.1, (0, 0, 0)),
          3: ("velocity", 0.9, (0, 0.02, 0)), 4: ("pressure", 1.0, (0.01, 0, 0))}
    want = oracle.run_ts(f0, solid, 7, 1.3, (1e-5, 0, 0))
    got = oracle.run_ts(f0, m, 7, 1.3, (1e-5, 0, 0), bc=bc)
    assert np.array_equal(got, want)


def test_golden_steady_96cube_starts_as_the_oracle_runs():
    """tests/golden/steady_96cube.txt was written by make_steady_96cube.py from the oracle alone: its
    pack and its first window's mean velocity are what the oracle computes now (bit for bit)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "steady_96cube.txt")
    vals, hist = {}, {}
    for line in open(path):
        f = line.split("#", 1)[0].split()
        if not f:
            continue
        if f[0] == "U_at":
            hist[int(f[1])] = float(f[2])
        else:
            vals[f[0]] = f[1]
    n, g, omega, K = int(vals["lattice"]), float(vals["g"]), float(vals["omega"]), int(vals["K"])
    solid, spheres = lbm_inputs.sphere_pack(n, int(vals["radius"]), float(vals["porosity_target"]), int(vals["seed"]))
    assert spheres == int(vals["spheres"]) and int((solid == 0).sum()) == int(vals["n_fluid"])
    f = oracle.init_equilibrium(lbm_inputs.rho_u_field(solid.shape), solid)
    f = oracle.run_ts(f, solid, K, omega, (g, 0.0, 0.0))
    u = float(oracle.mean_velocity(oracle.moments(f, solid), (g, 0.0, 0.0))[0])
    assert u == hist[K]
    # the stored result follows from its last window by Darcy's law
    nu = (1.0 / omega - 0.5) / 3.0
    phi = int(vals["n_fluid"]) / solid.size
    assert abs(float(vals["permeability"]) - nu * phi * hist[int(vals["steps"])] / g) <= 1e-12 * float(vals["permeability"])
    # and the stop rule held: three windows under the stated tolerance
    s = int(vals["steps"])
    assert all(abs(hist[s - j * K] - hist[s - (j + 1) * K]) < float(vals["tol"]) * abs(hist[s]) for j in range(3))
