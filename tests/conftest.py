import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def g0():
    """The tiny plain-path workload: R-MAT scale 10, edge factor 16, 32 seeds."""
    import graphgen
    el = graphgen.rmat(10, 16, seed=1)
    seeds = graphgen.draw_seeds(el, 32, seed=7)
    return el, seeds


@pytest.fixture(scope="session")
def g0_oracle(g0):
    import oracle
    el, _ = g0
    return oracle.OracleGraph.from_edgelist(el)
