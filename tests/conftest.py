import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HARTREE_MEV = 27211.386245988


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def tiny_problem():
    from gwsynth import get_config, make_problem
    return make_problem(get_config("tiny"))


@pytest.fixture(scope="session")
def tiny_sos(tiny_problem):
    from oracle.g0w0 import g0w0_problem
    return g0w0_problem(tiny_problem, keep=True)


@pytest.fixture(scope="session")
def tiny_lt_grid(tiny_problem, tiny_sos):
    from oracle import grids
    c = tiny_problem.cfg
    lo, hi = grids.lt_bounds(tiny_problem.eps, c.n_fc, c.n_occ, tiny_sos.omega[0])
    x, w, err = grids.lt_grid(c.n_lt, lo, hi)
    return x, w, err, lo, hi


def two_level(r=0.3, p=0.4, q=0.2, e_i=-0.5, e_a=0.3):
    """One occupied i, one virtual a, one auxiliary function."""
    return dict(r=r, p=p, q=q, e_i=e_i, e_a=e_a)


@pytest.fixture
def rng():
    return np.random.default_rng(12345)
