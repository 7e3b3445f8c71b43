"""Seeded input generators: SplitMix64 test vector, sphere-pack definition and stop rule."""
import numpy as np
import pytest

import lbm_inputs


def test_splitmix64_published_first_outputs():
    # first three outputs of SplitMix64 seeded with 0 (the generator's reference sequence)
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [int(v) for v in lbm_inputs.splitmix64(0, 3)] == want
    st = lbm_inputs.SplitMix64(0)
    assert [st.next() for _ in range(3)] == want


def test_splitmix64_counter_form_matches_sequential():
    st = lbm_inputs.SplitMix64(12345)
    seq = [st.next() for _ in range(50)]
    assert [int(v) for v in lbm_inputs.splitmix64(12345, 40, start=10)] == seq[10:]


@pytest.mark.parametrize("n,r,phi,seed", [(12, 2, 0.6, 5), ((9, 7, 11), 3, 0.5, 8), (10, 4, 0.3, 1)])
def test_sphere_pack_matches_minimum_image_definition(n, r, phi, seed):
    m, cnt = lbm_inputs.sphere_pack(n, r, phi, seed)
    m2, cnt2 = lbm_inputs.sphere_pack_reference(n, r, phi, seed)
    assert cnt == cnt2
    np.testing.assert_array_equal(m, m2)


def test_sphere_pack_stops_at_first_sphere_reaching_target():
    m, cnt = lbm_inputs.sphere_pack(20, 3, 0.55, seed=4)
    assert 1 - m.mean() <= 0.55
    m_prev, _ = lbm_inputs.sphere_pack(20, 3, 0.55, seed=4, max_spheres=cnt - 1)
    assert 1 - m_prev.mean() > 0.55


def test_velocity_noise_order_and_range():
    u = lbm_inputs.velocity_noise((2, 3, 4), 1e-3, seed=1)
    U = lbm_inputs.uniform01(1, 3 * 24)
    # cell (x=1, y=0, z=0) is cell 1: its draws are 3, 4, 5 in the order x, y, z
    np.testing.assert_array_equal(u[:, 0, 0, 1], (2 * U[3:6] - 1) * 1e-3)
    assert np.abs(u).max() < 1e-3


def test_serving_request_ranges():
    seen = set()
    for s in range(200):
        p = lbm_inputs.serving_request(1000 + s)
        assert p["edge"] in range(32, 193, 16)
        assert 3 <= p["radius"] <= 10
        assert 0.3 <= p["porosity"] < 0.8
        seen.add(p["edge"])
    assert len(seen) == 11
