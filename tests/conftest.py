import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libfwbf.so")
    config.addinivalue_line("markers", "slow: long-running CPU test")


# codes of the workloads: (mb, nb, Z, seed)
CODES = {
    "n186": (3, 6, 31, 1),
    "n1008": (3, 6, 168, 2),
    "n4032": (3, 6, 672, 3),
    "n8000": (4, 20, 400, 4),
    "n32400": (3, 30, 1080, 5),
}


@pytest.fixture(scope="session")
def ocodes():
    import oracle
    cache = {}

    def get(name):
        if name not in cache:
            cache[name] = oracle.Code.from_seed(*CODES[name])
        return cache[name]
    return get
