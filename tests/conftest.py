import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def random_views(rng, n_views, radius=20.0, det_dist=20.0, pixel=1.0, allow_z=True):
    """Random cone-beam views around the origin: source on a sphere of the
    given radius, detector centre opposite, random in-plane orientation."""
    out = np.zeros((n_views, 12))
    for k in range(n_views):
        while True:
            w = rng.normal(size=3)
            w /= np.linalg.norm(w)
            if allow_z or abs(w[2]) < 0.6:
                break
        s = radius * w
        d = -det_dist * w
        a = rng.normal(size=3)
        a -= a.dot(w) * w
        a /= np.linalg.norm(a)
        b = np.cross(w, a)
        out[k, 0:3] = s
        out[k, 3:6] = d
        out[k, 6:9] = pixel * a
        out[k, 9:12] = pixel * b
    return out


@pytest.fixture
def rng():
    return np.random.Generator(np.random.PCG64(12345))
