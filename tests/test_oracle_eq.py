"""Pins of the oracle's EQ assembly: Appendix A's identities (element-wise
sums == global rho-masked assembly), the rho = 1 remark (Remark
rem:rom-eqp-ones), linearity in rho and invariance to the EQ list order."""
import numpy as np
import pytest

from conftest import rel
from oracle import assemble, eq
from oracle import residual as rs


def _rom(wl, el=None, rho=None):
    pb = rs.Problem(wl)
    return eq.ROM(pb, wl.Phi, wl.Psi, wl.eq_elem if el is None else el, wl.eq_rho if rho is None else rho)


@pytest.mark.parametrize("which", ["tiny", "euler_small", "st_burgers"])
def test_elementwise_equals_global_masked(which, request):
    wl = request.getfixturevalue(which)
    rom = _rom(wl)
    for k in (0, 3):
        mu, w, tau = wl.mus[k], wl.w_eval[k], wl.tau_eval[k]
        j = rom.jacobian(mu, w, tau)
        G = assemble.global_eq(rom.prob, mu, w, tau, wl.eq_elem, wl.eq_rho)
        assert abs(j["J"] - G["J"]) <= 1e-13 * abs(G["J"])
        assert rel(j["g"], G["g"]) < 1e-12
        assert rel(j["H"], G["H"]) < 1e-12
        r = rom.residual(mu, w, tau)
        assert rel(r["PhiT_r"], G["PhiT_r"]) < 1e-12
        assert abs(r["J"] - j["J"]) <= 1e-14 * j["J"]
        # stacked least-squares rows reproduce J~, g, H
        assert abs(0.5 * j["Ft"] @ j["Ft"] - j["J"]) <= 1e-13 * j["J"]
        assert rel(j["Jt"].T @ j["Ft"], j["g"]) < 1e-12
        assert rel(j["Jt"].T @ j["Jt"], j["H"]) < 1e-12


def test_rho_one_over_all_elements_gives_unweighted_rom(euler_small):
    """rho = 1: PhiT_r = Phi^T R, and g = [Phi^T R_U^T R; Psi^T (R_x^T R + N_x^T N)]."""
    wl = euler_small
    Ne = wl.mesh.n_elem
    rom = _rom(wl, np.arange(Ne), np.ones(Ne))
    mu, w, tau = wl.mus[2], wl.w_eval[2], wl.tau_eval[2]
    A = assemble.global_assemble(rom.prob, mu, wl.Phi @ w, wl.X + wl.Psi @ tau)
    R, N = A["R"], A["N"]
    r = rom.residual(mu, w, tau)
    assert rel(r["PhiT_r"], wl.Phi.T @ R) < 1e-12
    j = rom.jacobian(mu, w, tau)
    S = wl.Phi.T @ (A["RU"].T @ R)
    T = wl.Psi.T @ (A["Rx"].T @ R + A["Nx"].T @ N)
    assert rel(j["g"], np.r_[S, T]) < 1e-12
    assert abs(j["J"] - 0.5 * (R @ R + N @ N)) < 1e-13 * j["J"]


def test_linear_in_rho_and_order_invariant(tiny):
    wl = tiny
    mu, w, tau = wl.mus[4], wl.w_eval[4], wl.tau_eval[4]
    r1 = _rom(wl).jacobian(mu, w, tau)
    r2 = _rom(wl, rho=2.5 * wl.eq_rho).jacobian(mu, w, tau)
    assert rel(r2["g"], 2.5 * r1["g"]) < 1e-13 and rel(r2["H"], 2.5 * r1["H"]) < 1e-13
    perm = np.random.default_rng(5).permutation(wl.n_s)
    r3 = _rom(wl, wl.eq_elem[perm], wl.eq_rho[perm]).jacobian(mu, w, tau)
    assert rel(r3["g"], r1["g"]) < 1e-13 and rel(r3["H"], r1["H"]) < 1e-13
    # a duplicated element with weights r1 + r2 equals one entry with r1 + r2
    el = np.r_[wl.eq_elem, wl.eq_elem[:3]]
    rho = np.r_[wl.eq_rho, [0.3, 0.2, 0.1]]
    rho_m = wl.eq_rho.copy()
    rho_m[:3] += [0.3, 0.2, 0.1]
    r4 = _rom(wl, el, rho).jacobian(mu, w, tau)
    r5 = _rom(wl, rho=rho_m).jacobian(mu, w, tau)
    assert rel(r4["g"], r5["g"]) < 1e-13 and abs(r4["J"] - r5["J"]) < 1e-13 * r5["J"]
    # zero weight contributes nothing
    rho0 = wl.eq_rho.copy()
    rho0[0] = 0.0
    r6 = _rom(wl, rho=rho0).jacobian(mu, w, tau)
    r7 = _rom(wl, wl.eq_elem[1:], wl.eq_rho[1:]).jacobian(mu, w, tau)
    assert rel(r6["H"], r7["H"]) < 1e-13


def test_reduced_jacobian_matches_fd_of_stacked_residual(tiny, euler_small):
    """d F~ / d z by central differences equals J~_z (rows sqrt(rho)[A B; 0 a])."""
    for wl in (tiny, euler_small):
        rom = _rom(wl)
        mu, w, tau = wl.mus[6], wl.w_eval[6], wl.tau_eval[6]
        j = rom.jacobian(mu, w, tau)
        z = np.r_[w, tau]
        n = wl.n
        Jfd = np.zeros_like(j["Jt"])
        for i in range(z.size):
            h = 1e-6 * max(1.0, abs(z[i]))
            zp, zm = z.copy(), z.copy()
            zp[i] += h
            zm[i] -= h
            Jfd[:, i] = (rom.residual(mu, zp[:n], zp[n:])["Ft"] - rom.residual(mu, zm[:n], zm[n:])["Ft"]) / (2 * h)
        assert rel(j["Jt"], Jfd) < 1e-6


def test_gathers_are_rows_of_the_bases(euler_small):
    wl = euler_small
    rom = _rom(wl)
    pb = rom.prob
    for k, e in enumerate(wl.eq_elem):
        assert np.array_equal(rom.Phi_s[k], wl.Phi[e * 24:(e + 1) * 24])
        for f in range(3):
            E = wl.mesh.elem_nbr[e, f]
            blk = rom.Phin_s[k, f * 12:(f + 1) * 12]
            if E < 0:
                assert not blk.any()
            else:
                rows = pb.P_n[e, f * 12:(f + 1) * 12]
                assert (rows // 24 == E).all()
                assert np.array_equal(blk, wl.Phi[rows])
