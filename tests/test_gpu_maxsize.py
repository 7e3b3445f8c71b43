"""The largest box the library accepts (just under 2^31 cells), where 32-bit node
and block indices are closest to their limits.

FP16 shifted storage (81 GB) so that the lattice fits one MI355X.  Fully
periodic, so the exact laws of the collision hold for the whole box: mass is
conserved and the raw momentum grows by M g per step (the Guo force term adds
rho g to every node).  Both are read through the FP64 reduction.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_largest_direct_grid_conserves_mass_and_gains_momentum():
    import paper_1111_0922_amd as P
    nx, ny, nz = 2048, 1024, 1023          # 2,145,386,496 cells < 2^31
    g = 1e-6
    torch.cuda.empty_cache()
    grid = P.Grid(nx, ny, nz, precision="f16s", omega=1.2, g=(g, 0.0, 0.0), f16_scale=1024.0)
    assert grid.n_nodes == nx * ny * nz
    grid.bind("aa")
    grid.init_equilibrium()
    m0 = grid.moments().cpu().numpy()
    assert abs(m0[0] / grid.n_nodes - 1.0) <= 1e-12 and np.all(m0[1:] == 0.0)
    grid.step(2)                           # both AA kernels over every node
    m = grid.moments().cpu().numpy()
    # mass: the rest population closes the balance per node; what remains is the
    # binary16 rounding of the stored deviations (~1e-7 / sigma per node)
    assert abs(m[0] - m0[0]) / m0[0] <= 1e-8
    # momentum: 2 M g from rest, within the binary16 resolution of the increments (~1e-3)
    assert abs(m[1] - 2 * m0[0] * g) / (2 * m0[0] * g) <= 1e-2
    assert abs(m[2]) <= 1e-3 * 2 * m0[0] * g and abs(m[3]) <= 1e-3 * 2 * m0[0] * g
    del grid
    torch.cuda.empty_cache()


def _max_mask(nx, ny, nz):
    """uint8 [nz, ny, nx] on the device: fluid (0) where (3x + 5y + 7z) mod 11 < 3, solid (1) elsewhere
    (about 27% fluid, rows of uneven fluid runs), built plane by plane."""
    mask = torch.empty((nz, ny, nx), dtype=torch.uint8, device="cuda")
    x = torch.arange(nx, device="cuda", dtype=torch.int64)
    y = torch.arange(ny, device="cuda", dtype=torch.int64)
    xy = (3 * x[None, :] + 5 * y[:, None]) % 11
    for z in range(nz):
        mask[z] = ((xy + 7 * z) % 11 >= 3).to(torch.uint8)
    return mask


def test_largest_indirect_grid_rank_lookup_and_blocks_match_idx_and_plain_soa():
    """An indirect grid of just under 2^31 cells (5.8e8 fluid nodes), FP64, fully periodic: the default
    path (neighbour ids by rank, 1024-node blocks) and the IDX path in plain SoA give the same moments
    bit for bit after an even and an odd AA step, and mass is conserved.  Cell indices, ranks and
    blocked slot indices are then near their 32-bit limits."""
    import paper_1111_0922_amd as P
    nx, ny, nz = 2048, 1024, 1023
    torch.cuda.empty_cache()
    mask = _max_mask(nx, ny, nz)
    nf_want = int((mask == 0).sum().item())
    grid = P.Grid(nx, ny, nz, addressing="indirect", precision="f64", omega=1.2, g=(1e-6, 0.0, 0.0))
    assert grid.build_idx(mask) == nf_want
    del mask
    grid.cellmap = None
    grid._mask = None
    torch.cuda.empty_cache()
    out = []
    for rank, block in ((-1, -1), (0, 0)):
        grid.set_option(P._lib.OPT_RANK_LOOKUP, rank)
        grid.set_option(P._lib.OPT_SOA_BLOCK, block)
        grid.bind("aa")
        assert grid.rank_lookup == (rank != 0)
        grid.init_equilibrium()
        m0 = grid.moments().cpu().numpy()
        grid.step(2)
        m = grid.moments().cpu().numpy()
        assert abs(m[0] - m0[0]) / m0[0] <= 1e-12
        out.append(m)
        grid.buffers = None
        torch.cuda.empty_cache()
    assert np.array_equal(out[0].view(np.int64), out[1].view(np.int64))
    del grid
    torch.cuda.empty_cache()
