"""Pins of the oracle's snapshot alignment (eq. (align0)) and Gram-Schmidt
basis update (eq. (greedy1)), Section 3.3."""
import numpy as np
import pytest

import synth
from conftest import rel
from oracle import align
from oracle import physics as ph
from oracle import residual as rs


@pytest.fixture(scope="module")
def tiny_align():
    wl = synth.tiny_burgers()
    pb = rs.Problem(wl)
    Phi_j = wl.Phi[:, :3]
    return wl, pb, Phi_j


def _point(wl, Phi_j, k=0):
    w = Phi_j.T @ (wl.Phi @ wl.w_eval[k])
    x = wl.X + wl.Psi @ wl.tau_eval[k]
    return w, x


def test_jacobian_matches_central_fd(tiny_align):
    # dF/d(w, x) = [R_U Phi_j R_x; 0 N_x] against central differences of F in
    # every w direction and in a sample of node coordinates (x-coordinates of
    # all nodes not on a horizontal boundary edge: there the Lax-Friedrichs
    # speed ties and d/dy is one-sided, as in the element pins)
    wl, pb, Phi_j = tiny_align
    mu = wl.mus[0]
    w, x = _point(wl, Phi_j)
    F, invalid, A = align.residual(pb, Phi_j, mu, w, x)
    assert not invalid
    J = align.jacobian(pb, Phi_j, A)
    j = Phi_j.shape[1]
    rng = np.random.default_rng(7)
    cols = list(range(j)) + list(j + 2 * rng.choice(x.size // 2, 12, replace=False))
    for c in cols:
        z = np.r_[w, x]
        h = 1e-6 * max(1.0, abs(z[c]))
        zp, zm = z.copy(), z.copy()
        zp[c] += h
        zm[c] -= h
        Fp = align.residual(pb, Phi_j, mu, zp[:j], zp[j:])[0]
        Fm = align.residual(pb, Phi_j, mu, zm[:j], zm[j:])[0]
        fd = (Fp - Fm) / (2 * h)
        assert rel(J[:, c], fd) < 1e-6, c


def test_direction_is_the_bruteforce_least_squares_step(tiny_align):
    # the step solves min |J d + F|^2 + lambda |d_x|^2: compare with lstsq on
    # the FD Jacobian (all columns).  lambda > 0: rigid translations of all
    # nodes change neither R nor N here, so J has a null space, and a small
    # lambda amplifies the FD error in the near-null directions
    wl, pb, Phi_j = tiny_align
    mu = wl.mus[1]
    w, x = _point(wl, Phi_j, 1)
    j = Phi_j.shape[1]
    z = np.r_[w, x]
    F0 = align.residual(pb, Phi_j, mu, w, x)[0]
    Jfd = np.zeros((F0.size, z.size))
    for c in range(z.size):
        h = 1e-6 * max(1.0, abs(z[c]))
        zp, zm = z.copy(), z.copy()
        zp[c] += h
        zm[c] -= h
        Jfd[:, c] = (align.residual(pb, Phi_j, mu, zp[:j], zp[j:])[0]
                     - align.residual(pb, Phi_j, mu, zm[:j], zm[j:])[0]) / (2 * h)
    # the y-coordinates of nodes on horizontal boundary edges sit on the
    # Lax-Friedrichs tie (one-sided derivative): those columns are the
    # analytic ones, every other column is the difference quotient
    yn = wl.mesh.X[:, 1]
    on_h = np.nonzero((yn == yn.min()) | (yn == yn.max()))[0]
    masked = j + 2 * on_h + 1
    J = align.jacobian(pb, Phi_j, align.residual(pb, Phi_j, mu, w, x)[2])
    Jfd[:, masked] = J[:, masked]
    for lam in (1e-2, 1.0):
        dw, dx, _ = align.direction(pb, Phi_j, mu, w, x, lam)
        M = np.vstack([Jfd, np.hstack([np.zeros((x.size, j)), np.sqrt(lam) * np.eye(x.size)])])
        ref = np.linalg.lstsq(M, -np.r_[F0, np.zeros(x.size)], rcond=None)[0]
        assert rel(np.r_[dw, dx], ref) < 1e-4, lam


def test_aligned_free_stream_is_a_fixed_point():
    # U = the inflow state everywhere on the unmapped mesh: R = 0 (free stream)
    # and N = 0, so F = 0 and the step is zero
    wl = synth.tiny_burgers()
    pb = rs.Problem(wl)
    mu = wl.mus[0]
    ub = ph.burgers_inflow(mu, wl.bc_mu_scale)
    Phi_j = np.ones((wl.N_u, 1)) / np.sqrt(wl.N_u)
    w = np.array([ub * np.sqrt(wl.N_u)])
    dw, dx, d = align.direction(pb, Phi_j, mu, w, wl.X.copy(), 1e-3)
    assert d["J"] < 1e-26
    assert np.abs(dw).max() < 1e-12 and np.abs(dx).max() < 1e-12


def test_steps_decrease_the_objective(tiny_align):
    wl, pb, Phi_j = tiny_align
    mu = wl.mus[2]
    w, x = _point(wl, Phi_j, 2)
    J0 = align.objective(pb, Phi_j, mu, w, x)
    for _ in range(3):
        w, x, info = align.step(pb, Phi_j, mu, w, x, lam=1e-3)
        assert info["status"] == "ok" and info["J_new"] < info["J_old"]
    assert align.objective(pb, Phi_j, mu, w, x) < J0


def test_gram_schmidt_append():
    rng = np.random.default_rng(3)
    B = np.linalg.qr(rng.standard_normal((50, 4)))[0]
    v = rng.standard_normal(50) + B @ rng.standard_normal(4) * 1e3   # mostly inside span(B)
    C = align.gram_schmidt_append(B, v)
    assert np.abs(C.T @ C - np.eye(5)).max() < 1e-13
    assert np.array_equal(C[:, :4], B)
    assert np.linalg.norm(v - C @ (C.T @ v)) < 1e-11 * np.linalg.norm(v)
