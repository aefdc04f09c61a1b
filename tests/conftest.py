import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def library():
    from paper_2503_11674_amd import netgen
    return netgen.make_library()


def with_clock(nl, lib, fail_frac=0.05):
    """Attach the clock period that makes floor(fail_frac * E) endpoints fail,
    derived from an oracle timing run (arrival times do not depend on it)."""
    from oracle import ref
    from paper_2503_11674_amd import netgen
    st = ref.sta(nl, lib, clock_period=0.0)
    nl["clock_period"] = np.float32(netgen.clock_period_for_fail_fraction(st["at"][ref.endpoint_pins(nl)], fail_frac))
    return nl
