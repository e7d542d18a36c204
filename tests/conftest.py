import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def load_tables():
    """The paper's Tables I/II for the (14,7) code, as {name: list of ints}."""
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", "tables_14_7.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, *vals = line.split()
            out[name] = [int(v) for v in vals]
    return out


@pytest.fixture(scope="session")
def tables():
    return load_tables()
