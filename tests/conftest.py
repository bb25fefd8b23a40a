import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def angle_deg(a, b, signed=False):
    """Angle between unit-vector fields (..., 3) in degrees; unsigned by default."""
    import numpy as np
    dot = (a * b).sum(-1)
    if not signed:
        dot = np.abs(dot)
    cr = np.linalg.norm(np.cross(a, b), axis=-1)
    return np.degrees(np.arctan2(cr, dot))


@pytest.fixture(scope="session")
def oracle():
    from oracle import oracle as o
    o.load()
    return o
