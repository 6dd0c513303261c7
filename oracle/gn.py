"""Levenberg-Marquardt / Gauss-Newton solver for the EQ problem (oracle; test infrastructure).

Section 3.1.3 of the paper: iterate z_{n+1} = z_n + alpha Delta z with the
step from the linear least-squares problem of eq. (levmarq-step),
    min | [F~; 0] + [J~_w J~_tau; 0 sqrt(lambda) I] Delta z |,
equivalently the normal equations of eq. (lmstep),
    (J~^T J~ + lambda diag(0, I)) Delta z = -[S~; T~],
and stop when |S~|_2 <= eps1 and |T~|_2 <= eps2 (eps1 = eps2 = 1e-8 in the
paper).  Readings: the step length comes from Armijo backtracking
(c1 = 1e-4, alpha halved from 1, at most 30 halvings), which enforces the
sufficient-decrease part of the Wolfe conditions the paper cites; lambda is a
caller parameter (0 = Gauss-Newton) because the paper's adaptive rule is in
a cited work; a trial point with invalid geometry or state has J~ = +inf.
"""
from __future__ import annotations

import numpy as np

from .eq import ROM


def lm_direction(jac, n, lam, solver="normal"):
    m = jac["H"].shape[0] - n
    if solver == "qr":
        A = np.vstack([jac["Jt"], np.hstack([np.zeros((m, n)), np.sqrt(lam) * np.eye(m)])])
        b = -np.r_[jac["Ft"], np.zeros(m)]
        return np.linalg.lstsq(A, b, rcond=None)[0]
    Hl = jac["H"].copy()
    Hl[n:, n:] += lam * np.eye(m)
    L = np.linalg.cholesky(Hl)
    y = np.linalg.solve(L, -jac["g"])
    return np.linalg.solve(L.T, y)


def gn_step(rom: ROM, mu, w, tau, lam=0.0, c1=1e-4, max_backtrack=30, tol=1e-8, solver="normal"):
    """One step from z_n = (w, tau).  Returns (w_new, tau_new, info).

    info: J_old, J_new, alpha, norm_S, norm_T (at z_n), n_backtrack,
    converged (z_n already meets the tolerance; no step taken), status
    ("ok", "converged", "linesearch", "singular", "invalid")."""
    n = rom.n
    jac = rom.jacobian(mu, w, tau)
    g = jac["g"]
    info = {"J_old": jac["J"], "J_new": jac["J"], "alpha": 0.0, "norm_S": float(np.linalg.norm(g[:n])),
            "norm_T": float(np.linalg.norm(g[n:])), "n_backtrack": 0, "converged": False, "status": "ok"}
    if not np.isfinite(jac["J"]):
        info["status"] = "invalid"
        return w, tau, info
    if info["norm_S"] <= tol and info["norm_T"] <= tol:
        info["converged"] = True
        info["status"] = "converged"
        return w, tau, info
    try:
        dz = lm_direction(jac, n, lam, solver)
    except np.linalg.LinAlgError:
        info["status"] = "singular"
        return w, tau, info
    slope = float(g @ dz)
    alpha = 1.0
    for bt in range(max_backtrack + 1):
        wt, tt = w + alpha * dz[:n], tau + alpha * dz[n:]
        Jt = rom.residual(mu, wt, tt)["J"]
        if Jt <= jac["J"] + c1 * alpha * slope:
            info.update(J_new=Jt, alpha=alpha, n_backtrack=bt)
            return wt, tt, info
        alpha *= 0.5
    info["status"] = "linesearch"
    info["n_backtrack"] = max_backtrack + 1
    return w, tau, info


def gn_solve(rom: ROM, mu, w0, tau0, tol=1e-8, max_it=50, **kw):
    w, tau = np.array(w0, dtype=float), np.array(tau0, dtype=float)
    hist = []
    for it in range(max_it + 1):
        w, tau, info = gn_step(rom, mu, w, tau, tol=tol, **kw)
        hist.append(info)
        if info["status"] != "ok":
            break
    return w, tau, hist
