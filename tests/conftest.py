import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle():
    from oracle import oracle as O
    O._lib()
    return O


@pytest.fixture(scope="session")
def workloads():
    from paper_2410_15227_amd import workloads as W
    W._lib()
    return W


@pytest.fixture(scope="session")
def uniform_4096(workloads):
    return workloads.uniform_4096(seed=1)


@pytest.fixture(scope="session")
def small_tess(workloads):
    """300 uniform generators, their particles and Voronoi grid."""
    pos, m, h, rho = workloads.make_cloud("uniform", 300, seed=11)
    return pos, m, h, workloads.voronoi(pos)


def rng(seed):
    return np.random.default_rng(seed)
