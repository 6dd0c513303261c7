import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="session")
def tiny():
    import synth
    return synth.tiny_burgers()


@pytest.fixture(scope="session")
def st_burgers():
    """The space-time Burgers problem with its source, 8x8 P1 cells."""
    import synth
    return synth.spacetime_burgers()


@pytest.fixture(scope="session")
def st_burgers_p2():
    """The space-time Burgers problem with its source, 4x4 P2 cells."""
    import synth
    return synth.spacetime_burgers(nx=4, ny=4, p=2, n=6, n_s=12)


@pytest.fixture(scope="session")
def euler_small():
    """8x4-cell P2 Euler mesh (64 elements), n = 20, m = 10, 12 EQ elements."""
    import synth
    return synth.euler_p2(nx=8, ny=4, n=20, m=10, n_s=12)


@pytest.fixture(scope="session")
def euler_mid():
    """16x8-cell P2 Euler mesh (256 elements), n = 20, m = 10, 64 EQ elements."""
    import synth
    return synth.euler_p2(nx=16, ny=8, n=20, m=10, n_s=64)
