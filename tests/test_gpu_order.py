"""Block-order tables of indirect grids: any permutation of the node blocks gives the same bits."""
import numpy as np
import pytest
import torch

import lbm_inputs
import oracle
from lbm_cases import from_device, make_grid, to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("scheme", ["aa", "ts", "os_push", "os_pull", "et"])
@pytest.mark.parametrize("layout", ["soa", "aos"])
def test_permuted_block_order_is_bit_identical(scheme, layout):
    import paper_1111_0922_amd as P
    solid = lbm_inputs.sphere_pack((40, 37, 33), 4, 0.5, seed=31)[0]
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=32))
    f0 = oracle.fluid_view(oracle.init_equilibrium(ru, solid), solid)
    out = []
    for permuted in (False, True):
        grid = make_grid(solid, scheme, addressing="indirect", layout=layout, omega=1.4, g=(1e-5, 0, 3e-6))
        nb = (grid.n_nodes + 255) // 256
        assert nb > 20
        if permuted:
            perm = np.random.default_rng(5).permutation(nb).astype(np.int32)
            grid.set_block_order(torch.from_numpy(perm).cuda())
        grid.set_pdfs(to_device(f0))
        grid.step(7)
        out.append((from_device(grid.get_pdfs()), from_device(grid.moments())))
    assert np.array_equal(out[0][0].view(np.int64), out[1][0].view(np.int64))
    assert np.array_equal(out[0][1], out[1][1])
    want = oracle.fluid_view(oracle.run_ts(oracle.init_equilibrium(ru, solid), solid, 7, 1.4, (1e-5, 0, 3e-6)), solid)
    assert float(np.max(np.abs(out[1][0] - want) / np.abs(want))) <= 1e-12


def test_block_order_validation():
    import paper_1111_0922_amd as P
    L = P._lib
    solid = lbm_inputs.sphere_pack(24, 3, 0.5, seed=2)[0]
    grid = make_grid(solid, "aa", addressing="indirect")
    nb = (grid.n_nodes + 255) // 256
    bad = torch.zeros(nb + 1, dtype=torch.int32, device="cuda")
    assert grid.lib.lbm_set_block_order(grid._h, ctypes_ptr(bad), nb + 1) == L.LBM_E_ARG
    direct = P.Grid(8, 8, 8)
    assert direct.lib.lbm_set_block_order(direct._h, ctypes_ptr(bad), nb) == L.LBM_E_UNSUPPORTED
    grid.set_block_order(None)


def ctypes_ptr(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())
