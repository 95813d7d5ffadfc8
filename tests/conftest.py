import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library on the device)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def kuhn2_jittered():
    import numpy as np
    from paper_2102_06248_amd import inputs
    xyz, tets = inputs.kuhn_cube(2)
    xyz = inputs.jitter_nodes(xyz, inputs.kuhn_interior_nodes(2), 0.5, 0.12, seed=7)
    return xyz, tets
