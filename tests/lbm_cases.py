"""Shared set-up of the GPU tests: building grids and moving canonical states."""
import numpy as np
import torch

import lbm_inputs
import oracle

SCHEMES = ["ts", "os_push", "os_pull", "aa", "et"]
LAYOUTS = ["soa", "aos"]
ADDRESSING = ["direct", "indirect"]
PRECISIONS = ["f64", "f32", "f16s", "f32s"]


def make_grid(solid, scheme, *, addressing="direct", layout="soa", precision="f64", omega=1.0,
              g=(0.0, 0.0, 0.0), f16_scale=1.0, wall_z=None, brick=None, trt_lambda=3.0 / 16.0):
    """Grid whose fluid nodes are the fluid cells of `solid` (uint8[nz, ny, nx]).

    Direct grids support a fully periodic box or the channel (solid planes
    z = 0 and z = nz - 1); indirect grids take the mask as it is.
    """
    import paper_1111_0922_amd as P
    nz, ny, nx = solid.shape
    if addressing == "direct":
        if wall_z is None:
            wall_z = bool(solid[0].all() and solid[-1].all() and nz >= 3 and not solid[1:-1].any())
        if not wall_z:
            assert not solid.any(), "direct grids hold a periodic box or a channel"
    grid = P.Grid(nx, ny, nz, addressing=addressing, layout=layout, precision=precision,
                  wall_z=bool(wall_z) if addressing == "direct" else False,
                  et_ghosts=(scheme == "et"), omega=omega, g=g, f16_scale=f16_scale, brick=brick,
                  trt_lambda=trt_lambda)
    if addressing == "indirect":
        grid.build_idx(torch.from_numpy(np.ascontiguousarray(solid, dtype=np.uint8)).cuda())
    grid.bind(scheme)
    return grid


def to_device(canon):
    return torch.from_numpy(np.ascontiguousarray(canon)).cuda()


def from_device(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def dense_from_canon(canon, solid):
    """float64[19, nz, ny, nx] with the node values at the fluid cells, zeros elsewhere."""
    f = np.zeros((19,) + solid.shape)
    f.reshape(19, -1)[:, solid.reshape(-1) == 0] = canon
    return f


def config1():
    """32^3 channel, walls z = 0 and 31, omega = 1, g = 1e-6 x, equilibrium with +-1e-3 noise (seed 1)."""
    solid = lbm_inputs.channel_mask(32, 32, 32)
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=1))
    f0 = oracle.init_equilibrium(ru, solid)
    return solid, f0, 1.0, (1e-6, 0.0, 0.0)


def rel_err(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))
