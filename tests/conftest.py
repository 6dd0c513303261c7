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


def rel_blocks(a, b, nblk):
    """Largest per-block error of a against b, split into nblk equal blocks
    (elements): |a_k - b_k| / (|b_k| + 1e-3 max_k |b_k|).  A block at least
    1e-3 of the largest is checked relative to itself; smaller blocks (a
    residual that cancels to rounding, a boundary block) against 1e-3 of the
    largest block instead of the whole array's norm."""
    a = np.asarray(a, dtype=np.float64).reshape(nblk, -1)
    b = np.asarray(b, dtype=np.float64).reshape(nblk, -1)
    nb = np.linalg.norm(b, axis=1)
    floor = 1e-3 * nb.max() if nb.max() > 0 else 1.0
    return float(np.max(np.linalg.norm(a - b, axis=1) / (nb + floor)))


def gram_entry_err(H, g, Ho, go, Jo):
    """Per-entry errors of the Gauss-Newton matrix and gradient, each on its
    own scale: H = M^T M gives |H_ij| <= sqrt(H_ii H_jj), and g = M^T F
    gives |g_i| <= sqrt(H_ii) |F| with |F|^2 = 2 J."""
    d = np.sqrt(np.maximum(np.diag(Ho), 0.0))
    sH = np.outer(d, d)
    sg = d * np.sqrt(2.0 * Jo)
    eH = np.abs(np.asarray(H) - Ho) / np.where(sH > 0, sH, 1.0)
    eg = np.abs(np.asarray(g) - go) / np.where(sg > 0, sg, 1.0)
    return float(eH.max()), float(eg.max())


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
