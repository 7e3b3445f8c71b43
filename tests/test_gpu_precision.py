"""FP32 and FP16-shifted storage against the oracle with the same storage rounding.

The oracle computes each collision in FP64 and rounds the stored value to
the storage format; the GPU computes in FP32.  Tolerances follow from that:
  * FP32 storage: after one step a stored value may differ by the FP32
    arithmetic error of one collision (a few ulp of f, f ~ w_i <= 1/3):
    relative 1e-6 (16 ulp).  Over 100 steps the differences perturb the flow
    and grow like a random walk: relative 2e-5.
  * FP16 shifted storage h = (f - w_i) sigma: a stored code may round the
    other way when the FP32 and FP64 values straddle a rounding boundary, one
    binary16 ulp of h.  Here |f - w_i| < 2^-12, so |h| < 2^-12 sigma and one
    ulp of h is at most 2^-23 sigma, i.e. 2^-23 in f whatever sigma is.
    Bars: 4 such ulp (4.8e-7 in f) after one step, 8 after 100 steps.
Also checked: the reduced-precision runs stay within the stated distance of
the FP64 oracle, and mass stays conserved through the FP64 reduction.
"""
import numpy as np
import pytest

import oracle
from lbm_cases import ADDRESSING, LAYOUTS, config1, from_device, make_grid, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    solid, f0, omega, g = config1()
    f64_100 = oracle.fluid_view(oracle.run_ts(f0, solid, 100, omega, g), solid)
    return solid, f0, omega, g, f64_100


def _run(solid, scheme, precision, sigma, q0, steps, omega, g, addressing="direct", layout="soa"):
    grid = make_grid(solid, scheme, addressing=addressing, layout=layout, precision=precision, omega=omega, g=g,
                     f16_scale=sigma)
    grid.set_pdfs(to_device(oracle.fluid_view(q0, solid)))
    m0 = from_device(grid.moments())
    grid.step(steps)
    return from_device(grid.get_pdfs()), m0, from_device(grid.moments())


@pytest.mark.parametrize("scheme", ["aa", "et", "ts", "os_pull"])
@pytest.mark.parametrize("addressing", ADDRESSING)
def test_fp32_storage(case, scheme, addressing):
    solid, f0, omega, g, f64_100 = case
    q0 = oracle.quantize(f0, solid, "f32")
    for steps, bar in ((1, 1e-6), (100, 2e-5)):
        want = oracle.fluid_view(oracle.run_ts(q0, solid, steps, omega, g, precision="f32"), solid)
        got, m0, m1 = _run(solid, scheme, "f32", 1.0, q0, steps, omega, g, addressing)
        assert float(np.max(np.abs(got - want) / np.abs(want))) <= bar, steps
        # plain FP32 storage: rounding of f ~ w_i repeats at steady state, mass drifts slowly
        assert abs(m1[0] - m0[0]) / m0[0] <= 1e-6
    assert float(np.max(np.abs(got - f64_100) / f64_100)) <= 2e-5


@pytest.mark.parametrize("sigma", [1.0, 1024.0])
@pytest.mark.parametrize("scheme", ["aa", "et", "ts", "os_push"])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_fp16_shifted_storage(case, sigma, scheme, layout):
    solid, f0, omega, g, f64_100 = case
    q0 = oracle.quantize(f0, solid, "f16s", sigma)
    ulp = 2.0 ** -23
    for steps, k in ((1, 4), (100, 8)):
        want = oracle.fluid_view(oracle.run_ts(q0, solid, steps, omega, g, precision="f16s", sigma=sigma), solid)
        got, m0, m1 = _run(solid, scheme, "f16s", sigma, q0, steps, omega, g, layout=layout)
        assert float(np.max(np.abs(got - want))) <= k * ulp, steps
    # distance to the full FP64 run after 100 steps
    assert float(np.max(np.abs(got - f64_100) / f64_100)) <= (1e-5 if sigma == 1.0 else 1e-6)


def test_fp16_scale_improves_accuracy(case):
    solid, f0, omega, g, f64_100 = case
    errs = {}
    for sigma in (1.0, 1024.0):
        q0 = oracle.quantize(f0, solid, "f16s", sigma)
        got, _, _ = _run(solid, "aa", "f16s", sigma, q0, 100, omega, g)
        errs[sigma] = float(np.max(np.abs(got - f64_100)))
    assert errs[1024.0] < errs[1.0] / 4


@pytest.mark.parametrize("sigma", [1.0, 1024.0])
@pytest.mark.parametrize("scheme", ["aa", "et", "os_pull"])
@pytest.mark.parametrize("addressing", ADDRESSING)
def test_fp32_shifted_storage(case, sigma, scheme, addressing):
    """FP32 shifted storage h = (f - w_i) sigma: the stored code carries ~2^-24 of the deviation
    (|f - w_i| < 2^-12 here, so < 2^-36 in f); the FP32 arithmetic of the deviation form adds a
    few ulp of rho = 1 (2^-23) to the mass moment.  Bars: 2e-9 in f after one step, 2e-8 after
    100 steps, and 2e-7 relative to the full FP64 run."""
    solid, f0, omega, g, f64_100 = case
    q0 = oracle.quantize(f0, solid, "f32s", sigma)
    for steps, bar in ((1, 2e-9), (100, 2e-8)):
        want = oracle.fluid_view(oracle.run_ts(q0, solid, steps, omega, g, precision="f32s", sigma=sigma), solid)
        got, m0, m1 = _run(solid, scheme, "f32s", sigma, q0, steps, omega, g, addressing)
        assert float(np.max(np.abs(got - want))) <= bar, steps
        assert abs(m1[0] - m0[0]) / m0[0] <= 1e-9
    assert float(np.max(np.abs(got - f64_100) / f64_100)) <= 2e-7


# Stated bounds on the steady-state permeability of each storage form relative to FP64 (the same
# bounds the 384^3 precision study reports against).  FP64 itself: 1e-10 of the oracle.
PERMEABILITY_BOUNDS = {("f32", 1.0): 1e-2, ("f32s", 1.0): 1e-5, ("f16s", 1.0): 5e-3, ("f16s", 1024.0): 1e-4}


def _golden_steady():
    import os
    vals, hist = {}, {}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "steady_96cube.txt")
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if not line:
                continue
            if line[0] == "U_at":
                hist[int(line[1])] = float(line[2])
            else:
                vals[line[0]] = line[1]
    return vals, hist


def test_permeability_chain_96cube_against_oracle_steady_state():
    """The FP64 oracle's steady state of a 96^3 sphere pack (r = 8, porosity 0.6, as the 384^3
    precision workload; tests/golden/steady_96cube.txt, written by the oracle alone) against the
    GPU AA pattern on the indirect grid: FP64 follows the oracle's mean velocity window by window
    (1e-9) and ends at its permeability (1e-10); every reduced storage form, run with the same
    steady-state rule as the precision study (paper_1111_0922_amd.steady), reaches a steady state
    (converged, or at its rounding-noise floor) within its stated bound of the oracle."""
    import lbm_inputs
    from paper_1111_0922_amd.steady import SteadyMonitor
    vals, hist = _golden_steady()
    n, r, phi_t, seed = int(vals["lattice"]), int(vals["radius"]), float(vals["porosity_target"]), int(vals["seed"])
    omega, g, K = float(vals["omega"]), float(vals["g"]), int(vals["K"])
    solid, spheres = lbm_inputs.sphere_pack(n, r, phi_t, seed)
    nf = int((solid == 0).sum())
    assert spheres == int(vals["spheres"]) and nf == int(vals["n_fluid"])
    phi = nf / solid.size
    nu = (1.0 / omega - 0.5) / 3.0
    k_oracle = float(vals["permeability"])

    def mean_u(grid):
        m = from_device(grid.moments())
        return (m[1] + 0.5 * m[0] * g) / m[0]

    grid = make_grid(solid, "aa", addressing="indirect", precision="f64", omega=omega, g=(g, 0, 0))
    grid.init_equilibrium()
    for t in range(K, int(vals["steps"]) + 1, K):
        grid.step(K)
        u = mean_u(grid)
        assert abs(u - hist[t]) / abs(hist[t]) <= 1e-9, (t, u, hist[t])
    assert abs(nu * phi * u / g - k_oracle) / k_oracle <= 1e-10
    del grid
    report = {}
    for (precision, sigma), bound in PERMEABILITY_BOUNDS.items():
        grid = make_grid(solid, "aa", addressing="indirect", precision=precision, omega=omega, g=(g, 0, 0),
                         f16_scale=sigma)
        grid.init_equilibrium()
        mon, steps = SteadyMonitor(1e-7), 0
        while steps < 20000 and mon.status == "running":
            grid.step(K)
            steps += K
            mon.push(mean_u(grid))
        k = nu * phi * mon.history[-1] / g
        report[(precision, sigma)] = (mon.status, steps, (k - k_oracle) / k_oracle)
        assert mon.steady, (precision, sigma, mon.status, steps)
        assert abs(k - k_oracle) / k_oracle <= bound, (precision, sigma, k, k_oracle, report)
        del grid
    print("96^3 chain (status, steps, rel. error vs the FP64 oracle):", report)


@pytest.mark.parametrize("precision", ["f16s", "f32", "f32s", "f64"])
@pytest.mark.parametrize("scheme", ["ts", "os_push", "os_pull", "aa", "et"])
@pytest.mark.parametrize("shape,walls", [((32, 32, 32), True), ((2, 3, 5), False), ((4, 4, 2), False),
                                         ((64, 6, 5), True), ((512, 3, 4), True), ((256, 5, 3), False),
                                         ((1024, 2, 4), True), ((1536, 1, 3), False)])
def test_pair_kernels_bit_identical_to_one_node(precision, scheme, shape, walls):
    """Direct SoA grids with nx a power of two up to 512, or a multiple of 512 (row segments),
    can update two nodes per lane; one node per lane must give the same bits, and both follow
    the oracle."""
    import lbm_inputs
    import paper_1111_0922_amd as P
    nx, ny, nz = shape
    solid = lbm_inputs.channel_mask(nx, ny, nz) if walls else np.zeros((nz, ny, nx), np.uint8)
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=13))
    sigma = 256.0 if precision in ("f16s", "f32s") else 1.0
    q0 = oracle.init_equilibrium(ru, solid)
    if precision != "f64":
        q0 = oracle.quantize(q0, solid, precision, sigma)
    out = []
    for pair in (1, 0):
        grid = make_grid(solid, scheme, precision=precision, omega=1.7, g=(1e-5, 2e-5, 0), f16_scale=sigma)
        grid.set_option(P._lib.OPT_PAIR, pair)
        grid.set_pdfs(to_device(oracle.fluid_view(q0, solid)))
        grid.step(5)
        out.append(from_device(grid.get_pdfs()))
    assert np.array_equal(out[0].view(np.int64), out[1].view(np.int64))
    want = oracle.fluid_view(oracle.run_ts(q0, solid, 5, 1.7, (1e-5, 2e-5, 0),
                                           precision=None if precision == "f64" else precision, sigma=sigma), solid)
    if precision == "f16s":
        assert float(np.max(np.abs(out[0] - want))) <= 8 * 2.0 ** -23
    elif precision == "f64":
        assert float(np.max(np.abs(out[0] - want) / np.abs(want))) <= 1e-12
    else:
        assert float(np.max(np.abs(out[0] - want) / np.abs(want))) <= 5e-6  # 1e-6 per step


@pytest.mark.parametrize("precision", ["f16s", "f32s", "f32", "f64"])
@pytest.mark.parametrize("scheme", ["ts", "os_push", "os_pull", "aa", "et"])
@pytest.mark.parametrize("shape,walls", [((512, 2, 4), True), ((768, 2, 3), False), ((1024, 1, 4), True),
                                         ((384, 2, 4), True), ((300, 3, 3), False), ((257, 2, 3), True),
                                         ((100, 3, 4), True), ((6, 5, 7), True), ((3, 1, 1), False)])
def test_wide_row_segments_bit_identical_to_plain(precision, scheme, shape, walls):
    """nx a multiple of 256: each workgroup stages one row segment and its end lanes reach
    beyond it in global memory; any other nx (not a power of two up to 256): the workgroup's
    256 nodes span rows and reach neighbours outside it in global memory.  The plain one-node
    kernels give the same bits."""
    import lbm_inputs
    import paper_1111_0922_amd as P
    nx, ny, nz = shape
    solid = lbm_inputs.channel_mask(nx, ny, nz) if walls else np.zeros((nz, ny, nx), np.uint8)
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=17))
    sigma = 256.0 if precision in ("f16s", "f32s") else 1.0
    q0 = oracle.init_equilibrium(ru, solid)
    if precision != "f64":
        q0 = oracle.quantize(q0, solid, precision, sigma)
    out = []
    for staged in (1, 0):
        grid = make_grid(solid, scheme, precision=precision, omega=1.7, g=(1e-5, 2e-5, 3e-6), f16_scale=sigma)
        grid.set_option(P._lib.OPT_PAIR, 0)
        grid.set_option(P._lib.OPT_ROW_STAGE, staged)
        grid.set_pdfs(to_device(oracle.fluid_view(q0, solid)))
        grid.step(5)
        out.append(from_device(grid.get_pdfs()))
    assert np.array_equal(out[0].view(np.int64), out[1].view(np.int64))
    want = oracle.fluid_view(oracle.run_ts(q0, solid, 5, 1.7, (1e-5, 2e-5, 3e-6),
                                           precision=None if precision == "f64" else precision, sigma=sigma), solid)
    if precision == "f16s":
        assert float(np.max(np.abs(out[0] - want))) <= 8 * 2.0 ** -23
    elif precision == "f64":
        assert float(np.max(np.abs(out[0] - want) / np.abs(want))) <= 1e-12
    else:
        assert float(np.max(np.abs(out[0] - want) / np.abs(want))) <= 5e-6  # 1e-6 per step


@pytest.mark.parametrize("precision", ["f16s", "f32s", "f32"])
@pytest.mark.parametrize("scheme", ["aa", "et", "os_pull"])
@pytest.mark.parametrize("shape,walls", [((6, 5, 7), True), ((11, 3, 4), False), ((3, 1, 1), False)])
def test_reduced_precision_ragged_boxes(precision, scheme, shape, walls):
    """Direct boxes whose nx is not a power of two run the one-node kernels (no
    row staging, no pairs); they follow the oracle with the same storage rounding."""
    import lbm_inputs
    nx, ny, nz = shape
    solid = lbm_inputs.channel_mask(nx, ny, nz) if walls else np.zeros((nz, ny, nx), np.uint8)
    ru = lbm_inputs.rho_u_field(solid.shape, lbm_inputs.velocity_noise(solid.shape, 1e-3, seed=15))
    sigma = 256.0 if precision != "f32" else 1.0
    q0 = oracle.quantize(oracle.init_equilibrium(ru, solid), solid, precision, sigma)
    want = oracle.fluid_view(oracle.run_ts(q0, solid, 7, 1.3, (1e-5, 0, 2e-6), precision=precision, sigma=sigma),
                             solid)
    got, _, _ = _run(solid, scheme, precision, sigma, q0, 7, 1.3, (1e-5, 0, 2e-6))
    if precision == "f16s":
        assert float(np.max(np.abs(got - want))) <= 8 * 2.0 ** -23   # as in test_fp16_shifted_storage
    else:
        assert float(np.max(np.abs(got - want) / np.abs(want))) <= 5e-6  # 1e-6 per step, 7 steps
