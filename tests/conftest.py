import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU runs of the oracle")


@pytest.fixture(scope="session", autouse=True)
def _built_host_parts():
    """The oracle and the input generators are small C libraries; build them if absent."""
    import lbm_inputs
    import oracle
    oracle.build(force=False)
    lbm_inputs.build(force=False)
    yield


@pytest.fixture(autouse=True)
def _announce_gpu_case(request):
    """Name each GPU case on stderr before it runs, so a run that ends abruptly still says where."""
    if request.node.get_closest_marker("gpu") is not None:
        import sys as _sys
        _sys.stderr.write(f"\n[gpu case] {request.node.nodeid}\n")
        _sys.stderr.flush()
    yield
