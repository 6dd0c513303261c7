"""Planted mistakes in the oracle (on the CPU) must each fail a pin.

Each case patches one plausible error into the oracle for the duration of
the test and checks that an independent pin detects it: a transposed mapping
Jacobian, a wrong neighbour orientation in the gather, a flipped upwinding
sign, a wrong distortion exponent, a wrong source and a missing block of the
alignment Jacobian."""
import numpy as np

from conftest import rel
from oracle import assemble, eq, physdg, physics as ph
from oracle import residual as rs
from oracle.dual import stack


def test_transposed_mapping_jacobian_is_caught(euler_small, monkeypatch):
    wl = euler_small
    good_inv = rs._inv2

    def bad_inv(J):
        Ji, det = good_inv(J)
        return stack([stack([Ji[..., 0, 0], Ji[..., 1, 0]], -1), stack([Ji[..., 0, 1], Ji[..., 1, 1]], -1)], -2), det
    monkeypatch.setattr(rs, "_inv2", bad_inv)
    pb = rs.Problem(wl)
    U = wl.Phi @ wl.w_eval[0]
    x = wl.X + wl.Psi @ wl.tau_eval[0]
    R = rs.hdm_assemble(pb, wl.mus[0], U, x, jac=False)["R"]
    assert rel(R, physdg.physical_residual(wl, wl.mus[0], U, x)) > 1e-6


def test_wrong_neighbour_orientation_is_caught(tiny, monkeypatch):
    wl = tiny
    good = rs.gather_maps

    def bad(mesh, p, n_c):
        P_e, P_n, Q_e = good(mesh, p, n_c)
        P_n = P_n.reshape(P_n.shape[0], 3, p + 1, n_c)[:, :, ::-1].reshape(P_n.shape[0], -1)
        return P_e, P_n, Q_e
    monkeypatch.setattr(rs, "gather_maps", bad)
    pb = rs.Problem(wl)
    rom = eq.ROM(pb, wl.Phi, wl.Psi, wl.eq_elem, wl.eq_rho)
    mu, w, tau = wl.mus[0], wl.w_eval[0], wl.tau_eval[0]
    G = assemble.global_eq(pb, mu, w, tau, wl.eq_elem, wl.eq_rho)
    assert rel(rom.jacobian(mu, w, tau)["g"], G["g"]) > 1e-6


def test_flipped_upwinding_is_caught(monkeypatch):
    monkeypatch.setattr(ph, "harten_abs", lambda lam, delta: -1.0 * ph.absd(lam))
    v = np.array([1.5, 0.4])
    G = 1.4
    st = lambda rho: np.array([[rho, rho * v[0], rho * v[1], 1.0 / (G - 1) + 0.5 * rho * v @ v]])
    nt = np.array([[2.0, 0.0]])
    H = ph.euler_roe(st(1.0), st(2.3), nt, G).v
    assert np.abs(H - ph.euler_flux(st(1.0), G).v[0] @ nt[0]).max() > 1e-3


def test_wrong_distortion_exponent_is_caught(euler_small, monkeypatch):
    wl = euler_small
    good = rs._eta

    def bad(G, g, detJ0, wq, eps):
        nG2 = (G * G).sum(axis=-1).sum(axis=-1)
        r = nG2 / (g * g)           # exponent 2 instead of 2/d = 1
        return rs.ein("eq,eq->e", r * r, wq[None, :] * detJ0)
    monkeypatch.setattr(rs, "_eta", bad)
    pb = rs.Problem(wl)
    X = wl.X.reshape(-1, 2)
    xs = (1.7 * X).reshape(-1)
    N = rs.hdm_assemble(pb, wl.mus[0], wl.Phi @ wl.w_eval[0], xs, jac=False)["N"]
    assert np.abs(N).max() > 1e-3
    assert good is not bad


def test_source_at_reference_position_is_caught(st_burgers, monkeypatch):
    # a wrong source (here exp(-b x)) breaks the identity with plain DG on
    # the physical mesh, which evaluates s on its own
    wl = st_burgers
    good = ph.burgers_source
    U = wl.Phi @ wl.w_eval[0]
    x = wl.X + wl.Psi @ wl.tau_eval[0]
    pb = rs.Problem(wl)
    R_good = rs.hdm_assemble(pb, wl.mus[0], U, x, jac=False)["R"]
    assert rel(R_good, physdg.physical_residual(wl, wl.mus[0], U, x)) < 1e-13

    def bad(xphys, mu, amp):   # the exponent's sign flipped
        return good(xphys, np.array([mu[0], -mu[1]]), amp)
    monkeypatch.setattr(ph, "burgers_source", bad)
    R = rs.hdm_assemble(rs.Problem(wl), wl.mus[0], U, x, jac=False)["R"]
    assert rel(R, physdg.physical_residual(wl, wl.mus[0], U, x)) > 1e-6


def test_alignment_without_distortion_rows_is_caught(monkeypatch):
    # dropping the N_x rows of the alignment Jacobian (or misplacing the
    # R_U Phi_j block) breaks the central-difference pin of dF/d(w, x)
    import synth
    from oracle import align
    wl = synth.tiny_burgers()
    pb = rs.Problem(wl)
    Phi_j = wl.Phi[:, :3]
    good = align.jacobian

    def bad(prob, Phi, A):
        J = good(prob, Phi, A)
        J[-A["Nx"].shape[0]:, :] = 0.0
        return J
    monkeypatch.setattr(align, "jacobian", bad)
    mu = wl.mus[0]
    w = Phi_j.T @ (wl.Phi @ wl.w_eval[0])
    x = wl.X + wl.Psi @ wl.tau_eval[0]
    F, _, A = align.residual(pb, Phi_j, mu, w, x)
    J = align.jacobian(pb, Phi_j, A)
    c = 3 + 2 * 40            # x-coordinate of an interior node
    h = 1e-6
    xp, xm = x.copy(), x.copy()
    xp[c - 3] += h
    xm[c - 3] -= h
    fd = (align.residual(pb, Phi_j, mu, w, xp)[0] - align.residual(pb, Phi_j, mu, w, xm)[0]) / (2 * h)
    assert rel(J[:, c], fd) > 1e-3


def test_harten_fix_without_factor_two_is_caught(monkeypatch):
    # (lam^2 + delta^2) / delta instead of / (2 delta): the fix then jumps
    # to 2 delta at |lam| = delta, and doubles the entropy-wave dissipation
    # of a slow contact; both pins must fail
    import test_oracle_physics as top
    good = ph.harten_abs

    def bad(lam, delta):
        a = ph.absd(lam)
        fixed = (lam * lam + delta * delta) / (1.0 * delta)
        return ph.where(a.v < delta.v, fixed, a)
    monkeypatch.setattr(ph, "harten_abs", bad)
    import pytest
    with pytest.raises(AssertionError):
        top.test_harten_fix_is_c1_at_the_threshold()
    with pytest.raises(AssertionError):
        top.test_roe_flux_at_a_slow_contact_matches_hand_computation()
    assert good is not bad
