"""Reference triangle, Lagrange basis and quadrature (oracle; test infrastructure).

The paper discretises with a "standard nodal DG method" on simplices and a
degree-q Lagrange mapping on the same mesh (Section 2.3, Section 4.1 and 4.2)
without fixing nodes or quadrature.  Readings taken here:

* nodes: vertices (0,0), (1,0), (0,1), then for degree 2 the mid-edge nodes
  of edges 0, 1, 2 (edge f joins vertex f and vertex f+1 mod 3);
* Lagrange basis: obtained by inverting the Vandermonde matrix of the
  monomials {xi^a eta^b, a + b <= p} at the nodes (no closed form used);
* volume quadrature: degree 2p symmetric rules, the 3-point rule for p = 1 and
  the 6-point two-orbit rule for p = 2, whose points and weights are solved
  here from the moment equations by Newton's method;
* face quadrature: (p+1)-point Gauss-Legendre on s in [0, 1].
"""
from __future__ import annotations

from functools import lru_cache
from math import factorial

import numpy as np

VERTS = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])


def nodes(p: int) -> np.ndarray:
    pts = [VERTS[0], VERTS[1], VERTS[2]]
    if p == 2:
        for f in range(3):
            pts.append(0.5 * (VERTS[f] + VERTS[(f + 1) % 3]))
    elif p != 1:
        raise ValueError("p must be 1 or 2")
    return np.array(pts)


def _monomials(p: int):
    return [(a, b) for t in range(p + 1) for a in range(t, -1, -1) for b in [t - a]]


def _vander(p: int, pts: np.ndarray):
    mons = _monomials(p)
    xi, eta = pts[:, 0], pts[:, 1]
    V = np.stack([xi ** a * eta ** b for a, b in mons], axis=1)
    Vx = np.stack([(a * xi ** (a - 1) if a > 0 else 0 * xi) * eta ** b for a, b in mons], axis=1)
    Vy = np.stack([xi ** a * (b * eta ** (b - 1) if b > 0 else 0 * eta) for a, b in mons], axis=1)
    return V, Vx, Vy


@lru_cache(maxsize=None)
def _coef(p: int) -> np.ndarray:
    V, _, _ = _vander(p, nodes(p))
    return np.linalg.inv(V)


def basis(p: int, pts: np.ndarray):
    """phi [P, nn] and grad phi [P, nn, 2] at reference points pts [P, 2]."""
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    C = _coef(p)
    V, Vx, Vy = _vander(p, pts)
    return V @ C, np.stack([Vx @ C, Vy @ C], axis=-1)


def triangle_moment(a: int, b: int) -> float:
    """Exact integral of xi^a eta^b over the reference triangle."""
    return factorial(a) * factorial(b) / factorial(a + b + 2)


def _orbit(a: float) -> np.ndarray:
    """The three points with barycentric coordinates (a, a, 1 - 2a) permuted."""
    c = 1.0 - 2.0 * a
    return np.array([[a, a], [c, a], [a, c]])


@lru_cache(maxsize=None)
def volume_rule(p: int):
    """Points [Q, 2] and weights [Q] of the degree-2p rule (weights sum to 1/2)."""
    if p == 1:
        return _orbit(1.0 / 6.0), np.full(3, 1.0 / 6.0)
    if p != 2:
        raise ValueError("p must be 1 or 2")
    mons = [(a, b) for t in range(5) for a in range(t + 1) for b in [t - a]]
    rhs = np.array([triangle_moment(a, b) for a, b in mons])

    def resid(z):
        a1, w1, a2, w2 = z
        pts = np.vstack([_orbit(a1), _orbit(a2)])
        wts = np.r_[np.full(3, w1), np.full(3, w2)]
        return np.array([(wts * pts[:, 0] ** a * pts[:, 1] ** b).sum() for a, b in mons]) - rhs

    z = np.array([0.45, 0.11, 0.09, 0.055])
    for _ in range(50):
        r = resid(z)
        Jm = np.empty((len(mons), 4))
        for k in range(4):
            h = 1e-7
            zp = z.copy()
            zp[k] += h
            zm = z.copy()
            zm[k] -= h
            Jm[:, k] = (resid(zp) - resid(zm)) / (2 * h)
        dz = np.linalg.lstsq(Jm, -r, rcond=None)[0]
        z = z + dz
        if np.abs(dz).max() < 1e-17:
            break
    a1, w1, a2, w2 = z
    return np.vstack([_orbit(a1), _orbit(a2)]), np.r_[np.full(3, w1), np.full(3, w2)]


@lru_cache(maxsize=None)
def face_rule(p: int):
    """Gauss-Legendre points s [p+1] and weights (sum 1) on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(p + 1)
    return 0.5 * (x + 1.0), 0.5 * w


def face_points(f: int, s: np.ndarray) -> np.ndarray:
    """Reference points on edge f, parametrised from vertex f (s=0) to f+1 (s=1)."""
    a, b = VERTS[f], VERTS[(f + 1) % 3]
    s = np.asarray(s)[:, None]
    return (1.0 - s) * a + s * b


def edge_nodes(p: int, f: int):
    """Element node indices on edge f ordered by s (vertex f, [mid], vertex f+1)."""
    if p == 1:
        return [f, (f + 1) % 3]
    return [f, 3 + f, (f + 1) % 3]


def lagrange_1d(p: int, s: np.ndarray):
    """1-D Lagrange basis on nodes k/p, values [P, p+1]."""
    s = np.asarray(s, dtype=np.float64)
    xs = np.arange(p + 1) / p
    L = np.ones((s.size, p + 1))
    for k in range(p + 1):
        for j in range(p + 1):
            if j != k:
                L[:, k] *= (s - xs[j]) / (xs[k] - xs[j])
    return L
