import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


M_WILSON = -1.4          # Wilson mass of every configuration (s = -1 - m = 0.4)
DIMS_SMALL = (4, 4, 4, 4)


class Dense:
    """Dense Q at 4^4 and its spectral decomposition (built once per session)."""

    def __init__(self, U, m, dims):
        import oracle
        self.U, self.m, self.dims = U, m, dims
        self.Q = oracle.dirac.dense_Q(U, m, dims)
        self.lam, self.W = np.linalg.eigh(self.Q)
        self.order = np.argsort(np.abs(self.lam), kind="stable")


@pytest.fixture(scope="session")
def dense_random():
    import synthetic
    return Dense(synthetic.gauge_field(DIMS_SMALL), M_WILSON, DIMS_SMALL)


@pytest.fixture(scope="session")
def dense_cold():
    import synthetic
    return Dense(synthetic.cold_gauge(DIMS_SMALL), M_WILSON, DIMS_SMALL)


@pytest.fixture(scope="session")
def dense_tiny():
    """Random-link 2x2x2x4 lattice (dimension 384) for operator-form checks."""
    import synthetic
    return Dense(synthetic.gauge_field((2, 2, 2, 4), seed=77), M_WILSON, (2, 2, 2, 4))
