"""Pins of the oracle's Levenberg-Marquardt / Gauss-Newton solver (Section
3.1.3): the step equals a brute-force least-squares step, J~ never
increases, the normal-equation and QR forms agree, and a zero-residual
problem converges to its closed-form minimiser."""
import numpy as np

from conftest import rel
from oracle import eq, gn
from oracle import residual as rs


def _rom(wl):
    return eq.ROM(rs.Problem(wl), wl.Phi, wl.Psi, wl.eq_elem, wl.eq_rho)


def test_step_equals_bruteforce_lstsq(tiny):
    wl = tiny
    rom = _rom(wl)
    mu, w, tau = wl.mus[0], wl.w_eval[3], wl.tau_eval[3]
    n = wl.n
    z = np.r_[w, tau]
    F0 = rom.residual(mu, w, tau)["Ft"]
    Jfd = np.zeros((F0.size, z.size))
    for i in range(z.size):
        h = 1e-6 * max(1.0, abs(z[i]))
        zp, zm = z.copy(), z.copy()
        zp[i] += h
        zm[i] -= h
        Jfd[:, i] = (rom.residual(mu, zp[:n], zp[n:])["Ft"] - rom.residual(mu, zm[:n], zm[n:])["Ft"]) / (2 * h)
    lam = 0.3
    A = np.vstack([Jfd, np.hstack([np.zeros((wl.m, n)), np.sqrt(lam) * np.eye(wl.m)])])
    dz_bf = np.linalg.lstsq(A, -np.r_[F0, np.zeros(wl.m)], rcond=None)[0]
    jac = rom.jacobian(mu, w, tau)
    for solver in ("normal", "qr"):
        assert rel(gn.lm_direction(jac, n, lam, solver), dz_bf) < 1e-6


def test_gn_monotone_and_twenty_steps(tiny):
    wl = tiny
    rom = _rom(wl)
    mu = wl.mus[0]
    w0, t0 = eq.plain_start(wl, mu)
    w, tau, hist = gn.gn_solve(rom, mu, w0, t0, max_it=19)
    Js = [h["J_old"] for h in hist] + [hist[-1]["J_new"]]
    assert all(b <= a for a, b in zip(Js, Js[1:]))
    assert Js[-1] < 0.5 * Js[0]
    gnorm = [np.hypot(h["norm_S"], h["norm_T"]) for h in hist]
    assert gnorm[-1] < 1e-3 * gnorm[0]


def test_zero_residual_minimiser(euler_small):
    """Angle 0 with walls: the free stream is an exact discrete solution and
    lies in span(Phi), so w* = Phi^T U_fs with J~ = 0.  At the free stream R
    vanishes for every mapping and N is second order in the deformation, so
    the tau-block of J~ is zero there: w converges to w*, tau only to a
    point where the (quartic) distortion term meets the tolerance.
    All elements carry rho = 1 here: an EQ set without inflow elements has a
    residual that is homogeneous of degree one in U (Euler flux, walls,
    outflow), hence the spurious minimiser U -> 0; the paper likewise requires
    weighted elements on every boundary (remark closing Section 4.2)."""
    wl = euler_small
    Ne = wl.mesh.n_elem
    rom = eq.ROM(rs.Problem(wl), wl.Phi, wl.Psi, np.arange(Ne), np.ones(Ne))
    mu = wl.mus[0]
    w_star, t_star = eq.plain_start(wl, mu)
    assert rom.residual(mu, w_star, t_star)["J"] < 1e-26
    rng = np.random.default_rng(7)
    w0 = w_star + 0.5 * rng.standard_normal(wl.n)
    t0 = 0.2 * wl.tau_eval[0]
    w, tau, hist = gn.gn_solve(rom, mu, w0, t0, max_it=25)
    assert hist[-1]["status"] == "converged"
    assert rel(w, w_star) < 1e-8
    assert hist[-1]["J_old"] < 1e-9 * hist[0]["J_old"]
    Js = [h["J_old"] for h in hist]
    assert all(b <= a for a, b in zip(Js, Js[1:]))


def test_linesearch_rejects_invalid_trial(tiny):
    """A trial point that folds an element has J~ = +inf and is backtracked."""
    wl = tiny
    rom = _rom(wl)
    mu, w = wl.mus[0], wl.w_eval[0]
    r = rom.residual(mu, w, 80.0 * wl.tau_eval[0])
    assert r["invalid"] and np.isinf(r["J"])


def test_w_only_step_equals_bruteforce_lstsq(tiny):
    """The initialisation step (w with tau held): least squares in the w
    columns of a finite-difference Jacobian of F~, dtau = 0 exactly."""
    wl = tiny
    rom = _rom(wl)
    mu, w, tau = wl.mus[0], wl.w_eval[5], wl.tau_eval[5]
    n = wl.n
    F0 = rom.residual(mu, w, tau)["Ft"]
    Jfd = np.zeros((F0.size, n))
    for i in range(n):
        h = 1e-6 * max(1.0, abs(w[i]))
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        Jfd[:, i] = (rom.residual(mu, wp, tau)["Ft"] - rom.residual(mu, wm, tau)["Ft"]) / (2 * h)
    dw_bf = np.linalg.lstsq(Jfd, -F0, rcond=None)[0]
    jac = rom.jacobian(mu, w, tau)
    for solver in ("normal", "qr"):
        dz = gn.lm_direction(jac, n, 0.7, solver, w_only=True)   # lambda plays no part
        assert rel(dz[:n], dw_bf) < 1e-6
        assert np.all(dz[n:] == 0.0)


def test_presolve_holds_tau_and_meets_tolerance(tiny):
    """The paper's initialisation from tau0 = 0 ends at |S~(w0, 0)| <= tol
    with tau untouched; the full iteration then converges."""
    wl = tiny
    rom = _rom(wl)
    mu = wl.mus[0]
    w0, t0 = eq.plain_start(wl, mu)
    w, tau = w0.copy(), t0.copy()
    for _ in range(40):
        w, tau, info = gn.gn_step(rom, mu, w, tau, w_only=True)
        assert np.array_equal(tau, t0)
        if info["status"] != "ok":
            break
    assert info["status"] == "converged" and info["norm_S"] <= 1e-8
    # the same through lm_solve: the w steps end where the loop above ends
    w2, tau2, res = gn.lm_solve(rom, mu, w0, t0, presolve=True, max_it=80)
    assert res["status"] == "converged" and res["w_iterations"] >= 1
    J = rom.jacobian(mu, w2, tau2)
    assert np.linalg.norm(J["g"][:wl.n]) <= 1e-8 and np.linalg.norm(J["g"][wl.n:]) <= 1e-8


def test_adaptive_lambda_rule():
    assert gn.adapt_lambda(1e-3, 1.0) == 1e-4
    assert gn.adapt_lambda(5e-12, 1.0) == 0.0
    assert gn.adapt_lambda(1e-3, 0.5) == 1e-2
    assert gn.adapt_lambda(0.0, 0.25) == 1e-8
