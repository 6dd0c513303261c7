"""Fluxes, numerical fluxes and boundary states (oracle; test infrastructure).

Physical fluxes are the paper's: the space-time Burgers flux (u^2/2, u) of
eq. (burgers) with its source s(x; (a, b)) = s_0 exp(b x) (s_0 = 0.02 in the
paper; 0 switches it off), and the Euler flux of eq. (euler) with the
ideal-gas pressure P = (gamma-1)(rho E - rho |v|^2 / 2).  The paper does not
name its numerical fluxes; the readings here are a local Lax-Friedrichs flux
for Burgers and Roe's approximate Riemann solver with Harten's entropy fix
(delta = 0.1 times the Roe-averaged sound speed, applied to all four waves)
for Euler.  Every function works on NumPy arrays or on ``Dual`` arrays; the
conservative components are the last axis.  ``nt`` is the scaled (not unit)
outward normal, so every numerical flux is homogeneous of degree one in it.
"""
from __future__ import annotations

import numpy as np

from .dual import Dual, absd, exp, lift, maximum, sqrt, stack, where


def _nd(*xs):
    for x in xs:
        if isinstance(x, Dual):
            return x.nd
    return 0


# ------------------------------------------------------------------ Burgers
def burgers_flux(u):
    """f(u) = (u^2 / 2, u): [..., 1] -> [..., 1, 2]."""
    nd = _nd(u)
    u = lift(u, nd)[..., 0]
    return stack([stack([0.5 * u * u, u], axis=-1)], axis=-2)


def burgers_lf(uL, uR, nt):
    """Local Lax-Friedrichs: H = (f(uL) + f(uR)).nt / 2 - alpha (uR - uL) / 2,
    alpha = max(|f'(uL).nt|, |f'(uR).nt|) with f'(u) = (u, 1)."""
    nd = _nd(uL, uR, nt)
    uL, uR, nt = lift(uL, nd)[..., 0], lift(uR, nd)[..., 0], lift(nt, nd)
    nx, ny = nt[..., 0], nt[..., 1]
    fnL = 0.5 * uL * uL * nx + uL * ny
    fnR = 0.5 * uR * uR * nx + uR * ny
    a = maximum(absd(uL * nx + ny), absd(uR * nx + ny))
    H = 0.5 * (fnL + fnR) - 0.5 * a * (uR - uL)
    return stack([H], axis=-1)


# -------------------------------------------------------------------- Euler
def euler_primitives(u, gamma):
    nd = _nd(u)
    u = lift(u, nd)
    rho, mx, my, E = u[..., 0], u[..., 1], u[..., 2], u[..., 3]
    vx, vy = mx / rho, my / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (vx * vx + vy * vy))
    return rho, vx, vy, E, p


def euler_flux(u, gamma):
    """Eq. (euler): rows (rho v, rho v (x) v + P I, (rho E + P) v): [..., 4] -> [..., 4, 2]."""
    rho, vx, vy, E, p = euler_primitives(u, gamma)
    fx = stack([rho * vx, rho * vx * vx + p, rho * vy * vx, (E + p) * vx], axis=-1)
    fy = stack([rho * vy, rho * vx * vy, rho * vy * vy + p, (E + p) * vy], axis=-1)
    return stack([fx, fy], axis=-1)


def roe_waves(uL, uR, n, gamma):
    """Roe-averaged wave speeds, strengths and right eigenvectors for the
    unit normal n: returns (lams[4], alphas[4], rvecs[4] each [..., 4]) with
    sum_k lam_k alpha_k r_k = (f(uR) - f(uL)) . n (Roe's property)."""
    nd = _nd(uL, uR, n)
    uL, uR, n = lift(uL, nd), lift(uR, nd), lift(n, nd)
    rL, uxL, uyL, EL, pL = euler_primitives(uL, gamma)
    rR, uxR, uyR, ER, pR = euler_primitives(uR, gamma)
    nx, ny = n[..., 0], n[..., 1]
    HL = (EL + pL) / rL
    HR = (ER + pR) / rR
    sL, sR = sqrt(rL), sqrt(rR)
    den = sL + sR
    rt = sL * sR
    ut = (sL * uxL + sR * uxR) / den
    vt = (sL * uyL + sR * uyR) / den
    Ht = (sL * HL + sR * HR) / den
    q2 = ut * ut + vt * vt
    ct = sqrt((gamma - 1.0) * (Ht - 0.5 * q2))
    vn = ut * nx + vt * ny
    vtan = vt * nx - ut * ny
    dr = rR - rL
    dp = pR - pL
    dvn = (uxR * nx + uyR * ny) - (uxL * nx + uyL * ny)
    dvt = (uyR * nx - uxR * ny) - (uyL * nx - uxL * ny)
    c2 = ct * ct
    a1 = (dp - rt * ct * dvn) / (2.0 * c2)
    a4 = (dp + rt * ct * dvn) / (2.0 * c2)
    a2 = dr - dp / c2
    a3 = rt * dvt
    one = lift(np.ones_like(rt.v), rt.nd)
    zero = 0.0 * one
    r1 = stack([one, ut - ct * nx, vt - ct * ny, Ht - ct * vn], axis=-1)
    r2 = stack([one, ut, vt, 0.5 * q2], axis=-1)
    r3 = stack([zero, -1.0 * ny * one, nx * one, vtan], axis=-1)
    r4 = stack([one, ut + ct * nx, vt + ct * ny, Ht + ct * vn], axis=-1)
    lams = [vn - ct, vn, vn, vn + ct]
    return lams, [a1, a2, a3, a4], [r1, r2, r3, r4], ct


def harten_abs(lam, delta):
    """|lam| with Harten's C^1 entropy fix: (lam^2 + delta^2) / (2 delta) for |lam| < delta."""
    a = absd(lam)
    fixed = (lam * lam + delta * delta) / (2.0 * delta)
    return where(a.v < delta.v, fixed, a)


def euler_roe(uL, uR, nt, gamma):
    """H = (f(uL) + f(uR)).nt / 2 - |nt| sum_k |lam_k|_fix alpha_k r_k / 2."""
    nd = _nd(uL, uR, nt)
    uL, uR, nt = lift(uL, nd), lift(uR, nd), lift(nt, nd)
    nmag = sqrt(nt[..., 0] * nt[..., 0] + nt[..., 1] * nt[..., 1])
    n = stack([nt[..., 0] / nmag, nt[..., 1] / nmag], axis=-1)
    fL = euler_flux(uL, gamma)
    fR = euler_flux(uR, gamma)
    fnL = fL[..., 0] * nt[..., None, 0] + fL[..., 1] * nt[..., None, 1]
    fnR = fR[..., 0] * nt[..., None, 0] + fR[..., 1] * nt[..., None, 1]
    lams, alphas, rvecs, ct = roe_waves(uL, uR, n, gamma)
    delta = 0.1 * ct
    diss = None
    for lam, al, r in zip(lams, alphas, rvecs):
        term = r * (harten_abs(lam, delta) * al)[..., None]
        diss = term if diss is None else diss + term
    return 0.5 * (fnL + fnR) - 0.5 * diss * nmag[..., None]


# ----------------------------------------------------------- boundary states
def euler_free_stream(mu, gamma):
    """Free stream of Section 4.2: rho = 1, P = 1, c = sqrt(gamma), |v| = M c,
    with mu = (M, inflow angle in degrees)."""
    M = float(mu[0])
    a = np.deg2rad(float(mu[1])) if len(mu) > 1 else 0.0
    c = np.sqrt(gamma)
    return np.array([1.0, M * c * np.cos(a), M * c * np.sin(a), 1.0 / (gamma - 1.0) + 0.5 * gamma * M * M])


def burgers_inflow(mu, bc_mu_scale):
    return 1.0 + bc_mu_scale * float(mu[0])


def burgers_boundary_values(mu, params):
    """(u+ on tag 1, u+ on tag 3).  The space-time problem of eq. (burgers)
    (``bc_spacetime``) prescribes u(0, t) = a = mu[0] on the left edge and
    the initial state u(x, 0) = 1 on the bottom edge; otherwise both edges
    take the inflow value 1 + bc_mu_scale mu[0]."""
    if params.get("bc_spacetime", False):
        return float(mu[0]), 1.0
    ub = burgers_inflow(mu, params["bc_mu_scale"])
    return ub, ub


def burgers_source(xphys, mu, amp):
    """s(x; (a, b)) = amp exp(b x) of eq. (burgers) at the physical first
    coordinate x (array or Dual), b = mu[1]."""
    return amp * exp(float(mu[1]) * xphys)


def boundary_state(pde, tag, uL, nt, mu, params):
    """Exterior state on a boundary face with tag 1 (left), 2 (right),
    3 (bottom) or 4 (top).

    Burgers: tags 1 and 3 inflow (``burgers_boundary_values``); tags 2
    and 4 outflow u+ = u-.  Euler: tag 1 supersonic inflow u+ = U_inf(mu); tag 2
    supersonic outflow u+ = u-; tags 3 and 4 slip walls
    u+ = (rho, rho v - 2 (rho v . n) n, rho E) with n = nt / |nt|.
    With ``all_farfield`` every Euler tag takes u+ = U_inf(mu).
    """
    nd = _nd(uL, nt)
    uL = lift(uL, nd)
    if pde == "burgers":
        if tag in (1, 3):
            ub = burgers_boundary_values(mu, params)[0 if tag == 1 else 1]
            return lift(np.full(uL.shape, ub), nd)
        return uL
    gamma = params["gamma"]
    if params.get("all_farfield", False) or tag == 1:
        return lift(np.broadcast_to(euler_free_stream(mu, gamma), uL.shape).copy(), nd)
    if tag == 2:
        return uL
    nt = lift(nt, nd)
    nmag = sqrt(nt[..., 0] * nt[..., 0] + nt[..., 1] * nt[..., 1])
    nx, ny = nt[..., 0] / nmag, nt[..., 1] / nmag
    mn = uL[..., 1] * nx + uL[..., 2] * ny
    return stack([uL[..., 0], uL[..., 1] - 2.0 * mn * nx, uL[..., 2] - 2.0 * mn * ny, uL[..., 3]], axis=-1)


def flux(pde, u, params):
    return burgers_flux(u) if pde == "burgers" else euler_flux(u, params["gamma"])


def numerical_flux(pde, uL, uR, nt, params):
    return burgers_lf(uL, uR, nt) if pde == "burgers" else euler_roe(uL, uR, nt, params["gamma"])
