"""Two-relaxation-time collision on the GPU against the oracle's TRT and closed forms.

The paper's solver relaxes with TRT (Sec. 10).  Every scheme, addressing and
layout is compared with the oracle's independent TRT on a channel and on a
porous mask; the equal-rates case must reproduce the BGK kernel bit for bit;
at Lambda = 3/16 half-way bounce-back gives the exact Poiseuille parabola for
any w+, and away from it the slip follows (g/nu)(16 Lambda - 3)/24.
"""
import numpy as np
import pytest

import lbm_inputs
import oracle
from lbm_cases import ADDRESSING, LAYOUTS, PRECISIONS, SCHEMES, from_device, make_grid, rel_err, to_device

pytestmark = pytest.mark.gpu

C0 = np.array([0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0])


def _state(solid, seed):
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=seed))
    return oracle.init_equilibrium(ru, solid)


def _run_gpu(solid, f0, scheme, addressing, layout, omega, lam, g, steps, collider="trt", precision="f64"):
    grid = make_grid(solid, scheme, addressing=addressing, layout=layout, precision=precision, omega=omega,
                     g=g, trt_lambda=lam)
    grid.set_pdfs(to_device(oracle.fluid_view(f0, solid)))
    grid.step(steps, collider=collider)
    return from_device(grid.get_pdfs())


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("addressing", ADDRESSING)
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("omega,lam", [(1.6, 3.0 / 16.0), (0.9, 0.5)])
def test_trt_channel_matches_oracle(scheme, addressing, layout, omega, lam):
    solid = lbm_inputs.channel_mask(24, 20, 18)
    f0 = _state(solid, 21)
    g = (2e-6, -1e-6, 5e-7)
    steps = 13
    want = oracle.run_ts(f0, solid, steps, omega, g, collider="trt",
                         omega_minus=oracle.trt_omega_minus(omega, lam))
    got = _run_gpu(solid, f0, scheme, addressing, layout, omega, lam, g, steps)
    assert rel_err(got, oracle.fluid_view(want, solid)) <= 1e-12


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_trt_porous_matches_oracle(scheme, layout):
    solid = lbm_inputs.sphere_pack((30, 26, 22), 4, 0.55, 23)[0]
    f0 = _state(solid, 24)
    omega, lam, g = 1.3, 3.0 / 16.0, (1e-5, 0, 0)
    want = oracle.run_ts(f0, solid, 12, omega, g, collider="trt",
                         omega_minus=oracle.trt_omega_minus(omega, lam))
    got = _run_gpu(solid, f0, scheme, "indirect", layout, omega, lam, g, 12)
    assert rel_err(got, oracle.fluid_view(want, solid)) <= 1e-12


@pytest.mark.parametrize("precision", ["f32", "f32s", "f16s"])
@pytest.mark.parametrize("scheme", ["aa", "os_pull", "et"])
def test_trt_reduced_precision_matches_oracle(scheme, precision):
    """TRT with 4- and 2-byte storage against the oracle's TRT with the same storage rounding
    (FP32 collision on the GPU, FP64 in the oracle): the bars of the BGK storage tests."""
    import paper_1111_0922_amd as P
    solid = lbm_inputs.channel_mask(32, 12, 10)
    sigma = 256.0 if precision in ("f16s", "f32s") else 1.0
    omega, lam, g = 1.7, 0.5, (1e-5, 2e-5, 0)
    q0 = oracle.quantize(_state(solid, 27), solid, precision, sigma)
    want = oracle.fluid_view(oracle.run_ts(q0, solid, 5, omega, g, collider="trt",
                                           omega_minus=oracle.trt_omega_minus(omega, lam),
                                           precision=precision, sigma=sigma), solid)
    grid = make_grid(solid, scheme, precision=precision, omega=omega, g=g, f16_scale=sigma, trt_lambda=lam)
    grid.set_pdfs(to_device(oracle.fluid_view(q0, solid)))
    grid.step(5, collider="trt")
    got = from_device(grid.get_pdfs())
    if precision == "f16s":
        assert float(np.max(np.abs(got - want))) <= 8 * 2.0 ** -23
    else:
        assert float(np.max(np.abs(got - want) / np.abs(want))) <= 5e-6  # 1e-6 per step


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("scheme", ["aa", "ts"])
def test_trt_with_equal_rates_is_bgk_bitwise(scheme, precision):
    """Lambda = (1/w - 1/2)^2 gives w- = w (exactly, for these w): the TRT run is the BGK run."""
    solid = lbm_inputs.sphere_pack((20, 18, 16), 3, 0.6, 25)[0]
    f0 = _state(solid, 26)
    for omega in (1.0, 2.0 / 3.0, 0.5):
        lam = (1.0 / omega - 0.5) ** 2
        assert 1.0 / (lam / (1.0 / omega - 0.5) + 0.5) == omega
        a = _run_gpu(solid, f0, scheme, "indirect", "soa", omega, lam, (1e-5, 0, 0), 9, "trt", precision)
        b = _run_gpu(solid, f0, scheme, "indirect", "soa", omega, lam, (1e-5, 0, 0), 9, "bgk", precision)
        assert np.array_equal(a.view(np.int64), b.view(np.int64)), omega


def _poiseuille(addressing, omega, lam, nz=34, g=1e-6):
    nu = (1.0 / omega - 0.5) / 3.0
    H = nz - 2
    solid = lbm_inputs.channel_mask(2, 2, nz)
    grid = make_grid(solid, "aa", addressing=addressing, omega=omega, g=(g, 0, 0), trt_lambda=lam)
    grid.init_equilibrium()
    grid.step(int(5 * H * H / nu) // 2 * 2, collider="trt")
    f = from_device(grid.get_pdfs()).reshape(19, H, 2, 2)
    rho = f.sum(axis=0)
    ux = (np.tensordot(C0, f, axes=(0, 0)) + 0.5 * rho * g) / rho
    z = np.arange(1, nz - 1, dtype=np.float64)[:, None, None]
    exact = g / (2 * nu) * (z - 0.5) * (H + 0.5 - z)
    return ux, exact, nu, g


@pytest.mark.parametrize("addressing", ADDRESSING)
@pytest.mark.parametrize("omega", [0.8, 1.0, 1.7])
def test_trt_poiseuille_exact_at_lambda_3_16(addressing, omega):
    ux, exact, _, _ = _poiseuille(addressing, omega, 3.0 / 16.0)
    assert np.abs(ux - exact).max() / exact.max() < 1e-9


@pytest.mark.parametrize("lam", [0.05, 0.5])
def test_trt_poiseuille_slip_follows_lambda(lam):
    ux, exact, nu, g = _poiseuille("direct", 1.0, lam)
    slip = (ux - exact).mean()
    assert abs(slip / (g / nu * (16 * lam - 3) / 24) - 1) < 5e-3


def test_trt_needs_positive_lambda():
    import paper_1111_0922_amd as P
    solid = lbm_inputs.channel_mask(8, 8, 8)
    grid = make_grid(solid, "aa", trt_lambda=0.0)
    grid.init_equilibrium()
    with pytest.raises(P.LbmError):
        grid.step(1, collider="trt")
    grid.step(1, collider="bgk")
    assert grid.t == 1
