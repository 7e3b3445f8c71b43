"""Physics of the GPU path checked against closed forms, independently of the oracle.

Poiseuille flow between half-way bounce-back walls, driven by the Guo body
force: at the relaxation omega = 1/(1/2 + sqrt(3)/4) (BGK with Lambda = 3/16)
the discrete steady solution is the exact parabola u(z) = g/(2 nu) (z - 1/2)
(H + 1/2 - z) for fluid planes z = 1..H, and the slit's Darcy permeability is
H^3/(12 nz) (1 + 1/(2 H^2)).  Checked on the direct channel and on the
indirect grid with the walls given as a mask, for several schemes.  A shear
wave in a periodic box decays at the lattice viscosity nu = (1/omega - 1/2)/3.
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


@pytest.mark.parametrize("omega,tol", [(1.0, 1e-5), (1.6, 3e-3)])
@pytest.mark.parametrize("axis", ["x", "z"])
@pytest.mark.parametrize("scheme,addressing", [("aa", "direct"), ("et", "direct"), ("ts", "direct"),
                                               ("os_pull", "direct"), ("aa", "indirect"), ("et", "indirect")])
def test_shear_wave_decays_at_the_lattice_viscosity(scheme, addressing, axis, omega, tol):
    """A transverse wave u = U sin(k s) e_t (s along x or z, L = 64) in a fully periodic box decays as
    exp(-nu k^2 t) with nu = (1/omega - 1/2)/3, to O(k^2) relative terms (the tolerances of the oracle's
    own test).  Along x the shifts go through the kernels' LDS staging; the direct grids use the default
    storage orders (1024-cell blocks for the two-step, one-step and esoteric-twist schemes), the indirect
    ones the rank lookup and blocks."""
    L = 64
    shape = (L, 2, 2) if axis == "x" else (2, 2, L)       # (nx, ny, nz)
    nx, ny, nz = shape
    solid = np.zeros((nz, ny, nx), np.uint8)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    s = (xx if axis == "x" else zz).reshape(-1).astype(np.float64)
    k = 2 * np.pi / L
    t = 1 if axis == "x" else 0                           # u_y(x) or u_x(z)
    rho_u = np.zeros((4, solid.size))
    rho_u[0] = 1.0
    rho_u[1 + t] = 1e-4 * np.sin(k * s)
    grid = make_grid(solid, scheme, addressing=addressing, omega=omega, g=(0, 0, 0))
    grid.init_equilibrium(torch.from_numpy(rho_u).cuda())

    def amplitude():
        f = from_device(grid.get_pdfs())
        u = np.tensordot(C[t], f, axes=(0, 0)) / f.sum(axis=0)
        return float((u * np.sin(k * s)).sum() * 2 / solid.size)

    grid.step(200)
    a1 = amplitude()
    grid.step(2000)
    a2 = amplitude()
    nu = (1.0 / omega - 0.5) / 3.0
    assert abs(-math.log(a2 / a1) / (k * k * 2000) / nu - 1) < tol
