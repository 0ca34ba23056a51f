import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU run (physical pins of the oracle)")


def golden(name):
    """Read tests/golden/<name>: 'key value rounding citation...' lines."""
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split(None, 3)
            out[parts[0]] = (float(parts[1]), float(parts[2]), parts[3] if len(parts) > 3 else "")
    return out


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import orc
    orc.build(force=False)
    return orc
