"""Stream-only steps are exact permutations, for every scheme, layout, addressing and precision.

With the identity collider a time step only moves stored values, so after k
steps the GPU state must equal, bit for bit, the oracle's two-step run with
the identity collider (itself pinned to an independent numpy permutation).
The canonical state is read back right after the upload, so the comparison
starts from values that the storage precision represents exactly.
"""
import zlib

import numpy as np
import pytest

import lbm_inputs
import oracle
from lbm_cases import ADDRESSING, LAYOUTS, PRECISIONS, SCHEMES, dense_from_canon, from_device, make_grid, to_device

pytestmark = pytest.mark.gpu


def _random_canon(nf, precision, rng):
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)[:, None]
    if precision == "f64":
        bits = rng.integers(0, 2 ** 63, size=(19, nf), dtype=np.int64)
        bits[:, ::7] |= np.int64(0x7FF0000000000001)  # NaN payloads travel too
        return bits.view(np.float64)
    if precision == "f32":
        return rng.standard_normal((19, nf)).astype(np.float32).astype(np.float64)
    return w + 1e-3 * rng.standard_normal((19, nf))


def _geometries():
    rng = np.random.default_rng(2)
    yield "channel_12x10x9", lbm_inputs.channel_mask(12, 10, 9)
    yield "periodic_7x5x6", np.zeros((6, 5, 7), np.uint8)
    # nx a power of two: direct SoA grids take the row-staged kernels
    yield "channel_16x6x7", lbm_inputs.channel_mask(16, 6, 7)
    yield "periodic_4x3x5", np.zeros((5, 3, 4), np.uint8)
    yield "periodic_1x4x3", np.zeros((3, 4, 1), np.uint8)
    yield "porous_13x11x10", (rng.random((10, 11, 13)) < 0.3).astype(np.uint8)


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("addressing", ADDRESSING)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_stream_only_is_permutation(scheme, addressing, layout, precision):
    rng = np.random.default_rng(zlib.crc32(f"{scheme}/{addressing}/{layout}/{precision}".encode()))
    for name, solid in _geometries():
        if addressing == "direct" and name.startswith("porous"):
            continue
        nf = int((solid == 0).sum())
        grid = make_grid(solid, scheme, addressing=addressing, layout=layout, precision=precision, f16_scale=4.0)
        assert grid.n_nodes == nf
        x0 = _random_canon(nf, precision, rng)
        grid.set_pdfs(to_device(x0))
        y0 = from_device(grid.get_pdfs())
        if precision in ("f64", "f32"):
            assert np.array_equal(y0.view(np.int64), x0.view(np.int64))  # exact round trip
        ref = dense_from_canon(y0, solid)
        for k in (1, 2, 3):
            grid.step(1, collider="identity")
            got = from_device(grid.get_pdfs())
            ref = oracle.run_ts(ref, solid, 1, 1.0, (0, 0, 0), collider="identity")
            want = oracle.fluid_view(ref, solid)
            assert np.array_equal(got.view(np.int64), want.view(np.int64)), (name, k)
