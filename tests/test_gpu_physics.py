"""Physics of the GPU path checked against closed forms, independently of the oracle.

Poiseuille flow between half-way bounce-back walls, driven by the Guo body
force: at the relaxation omega = 1/(1/2 + sqrt(3)/4) (BGK with Lambda = 3/16)
the discrete steady solution is the exact parabola u(z) = g/(2 nu) (z - 1/2)
(H + 1/2 - z) for fluid planes z = 1..H, and the slit's Darcy permeability is
H^3/(12 nz) (1 + 1/(2 H^2)).  Checked on the direct channel and on the
indirect grid with the walls given as a mask, for several schemes.
"""
import math

import numpy as np
import pytest
import torch

import lbm_inputs
from lbm_cases import from_device, make_grid

pytestmark = pytest.mark.gpu

C = np.array([[0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0],
              [0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1],
              [0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1]])


@pytest.mark.parametrize("scheme", ["aa", "et", "ts", "os_pull"])
@pytest.mark.parametrize("addressing", ["direct", "indirect"])
def test_poiseuille_exact_at_magic_relaxation(scheme, addressing):
    nz, g = 34, 1e-6
    omega = 1.0 / (0.5 + math.sqrt(3.0) / 4.0)
    nu = (1.0 / omega - 0.5) / 3.0
    H = nz - 2
    solid = lbm_inputs.channel_mask(2, 2, nz)
    grid = make_grid(solid, scheme, addressing=addressing, omega=omega, g=(g, 0, 0))
    grid.init_equilibrium()
    steps = int(5 * H * H / nu) // 2 * 2
    grid.step(steps)
    f = from_device(grid.get_pdfs()).reshape(19, H, 2, 2)
    rho = f.sum(axis=0)
    ux = (np.tensordot(C[0], f, axes=(0, 0)) + 0.5 * rho * g) / rho
    z = np.arange(1, nz - 1, dtype=np.float64)[:, None, None]
    exact = g / (2 * nu) * (z - 0.5) * (H + 0.5 - z)
    assert np.abs(ux - exact).max() / exact.max() < 1e-9
    m = from_device(grid.moments())
    U = (m[1] + 0.5 * m[0] * g) / m[0]
    k = nu * (H / nz) * U / g
    assert abs(k / (H ** 3 / (12.0 * nz) * (1 + 1.0 / (2 * H * H))) - 1) < 1e-9


@pytest.mark.parametrize("precision,nz,bound", [("f32s", 34, 1e-4), ("f16s", 10, 1e-2), ("f16s", 34, None)])
def test_poiseuille_reduced_precision(precision, nz, bound):
    """The shifted storage forms reach the parabola within their resolution.

    Per step the body force changes a node's deviation by about g/u = 8 nu / H^2
    of itself.  binary16 resolves 2^-11 ~ 5e-4 of a value: for H = 8 the change
    (~2e-2) is resolved and the profile is reached to 1e-2; for H = 32 it is
    ~1.1e-3, at the resolution, and increments round away (for any sigma): the
    profile stagnates several percent low.  The last case records that limit.
    """
    g = 1e-6
    omega = 1.0 / (0.5 + math.sqrt(3.0) / 4.0)
    nu = (1.0 / omega - 0.5) / 3.0
    H = nz - 2
    solid = lbm_inputs.channel_mask(2, 2, nz)
    grid = make_grid(solid, "aa", precision=precision, omega=omega, g=(g, 0, 0), f16_scale=1024.0)
    grid.init_equilibrium()
    grid.step(int(5 * H * H / nu) // 2 * 2 + 2000)
    f = from_device(grid.get_pdfs()).reshape(19, H, 2, 2)
    rho = f.sum(axis=0)
    ux = (np.tensordot(C[0], f, axes=(0, 0)) + 0.5 * rho * g) / rho
    z = np.arange(1, nz - 1, dtype=np.float64)[:, None, None]
    exact = g / (2 * nu) * (z - 0.5) * (H + 0.5 - z)
    err = np.abs(ux - exact).max() / exact.max()
    if bound is not None:
        assert err < bound
    else:
        assert 1e-2 < err < 0.2  # stagnation below the binary16 resolution, as derived above
