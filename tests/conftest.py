import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    # build what is missing (only then): the HIP library, the oracle, the generators
    from paper_1705_02257_amd.build import build_library
    build_library(force=False)
    import oracle
    import workloads
    oracle.build()
    workloads.build()


def golden_lines(name):
    """Non-comment, non-empty lines of a golden fixture file."""
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.lstrip().startswith("#")]


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def workloads_mod():
    import workloads
    workloads.build()
    return workloads
