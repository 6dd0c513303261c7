"""Pins of the oracle's reference element: closed-form integrals, published
quadrature constants and the Lagrange property."""
import json
import os

import numpy as np
import pytest

from oracle import refelem as re

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("p", [1, 2])
def test_volume_rule_exact_to_degree_2p(p):
    pts, w = re.volume_rule(p)
    for t in range(2 * p + 1):
        for a in range(t + 1):
            b = t - a
            got = (w * pts[:, 0] ** a * pts[:, 1] ** b).sum()
            assert abs(got - re.triangle_moment(a, b)) < 1e-16, (a, b)


def test_volume_rule_p2_not_exact_beyond_degree_4():
    pts, w = re.volume_rule(2)
    errs = [abs((w * pts[:, 0] ** a * pts[:, 1] ** (5 - a)).sum() - re.triangle_moment(a, 5 - a)) for a in range(6)]
    assert max(errs) > 1e-6


def test_volume_rule_p2_matches_published_constants():
    """Dunavant (1985), degree-4 six-point rule (weights normalised to area 1)."""
    with open(os.path.join(GOLDEN, "dunavant_deg4.json")) as f:
        ref = json.load(f)
    pts, w = re.volume_rule(2)
    a = sorted({round(float(v), 15) for v in pts[:, 0]})
    for orbit in ref["orbits"]:
        k = int(np.argmin([abs(pts[i, 0] - orbit["a"]) for i in range(6)]))
        assert abs(pts[k, 0] - orbit["a"]) < 2e-15
        assert abs(2.0 * w[k] - orbit["weight"]) < 2e-15
    assert len(a) == 4


@pytest.mark.parametrize("p", [1, 2])
def test_face_rule_exact_to_degree_2p_plus_1(p):
    s, w = re.face_rule(p)
    for k in range(2 * p + 2):
        assert abs((w * s ** k).sum() - 1.0 / (k + 1)) < 1e-15


@pytest.mark.parametrize("p", [1, 2])
def test_lagrange_basis(p):
    X = re.nodes(p)
    phi, dphi = re.basis(p, X)
    assert np.abs(phi - np.eye(len(X))).max() < 1e-14
    rng = np.random.default_rng(0)
    pts = rng.uniform(0, 0.5, (20, 2))
    phi, dphi = re.basis(p, pts)
    assert np.abs(phi.sum(axis=1) - 1).max() < 1e-14
    assert np.abs(dphi.sum(axis=1)).max() < 1e-13
    # reproduces every polynomial of degree <= p, e.g. xi^p + 2 eta - 1
    fn = lambda z: z[:, 0] ** p + 2 * z[:, 1] - 1
    assert np.abs(phi @ fn(X) - fn(pts)).max() < 1e-13


def test_edge_traces_use_edge_nodes_only():
    for p in (1, 2):
        s, _ = re.face_rule(p)
        for f in range(3):
            phi, _ = re.basis(p, re.face_points(f, s))
            off = [i for i in range(len(re.nodes(p))) if i not in re.edge_nodes(p, f)]
            assert np.abs(phi[:, off]).max() < 1e-14
            # along the edge the trace is the 1-D Lagrange basis on k/p
            L = re.lagrange_1d(p, s)
            assert np.abs(phi[:, re.edge_nodes(p, f)] - L).max() < 1e-14
