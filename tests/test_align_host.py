"""Host part of the mapping-basis update, eq. (greedy1) (no GPU needed)."""
import numpy as np
import pytest

from paper_2305_15661_amd.align import gram_schmidt_append


def test_gram_schmidt_append_orthonormal_and_spanning():
    rng = np.random.default_rng(11)
    B = np.linalg.qr(rng.standard_normal((40, 3)))[0]
    v = rng.standard_normal(40) + 1e4 * (B @ rng.standard_normal(3))   # nearly inside span(B)
    C = gram_schmidt_append(B, v)
    assert np.array_equal(C[:, :3], B)
    assert np.abs(C.T @ C - np.eye(4)).max() < 1e-13
    assert np.linalg.norm(v - C @ (C.T @ v)) < 1e-11 * np.linalg.norm(v)


def test_gram_schmidt_append_rejects_a_dependent_vector():
    B = np.eye(5)[:, :2]
    with pytest.raises(ValueError):
        gram_schmidt_append(B, 2.0 * B[:, 0] - B[:, 1])
