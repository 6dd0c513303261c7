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


def lm_direction(jac, n, lam, solver="normal", w_only=False):
    """Step of eq. (levmarq-step) / (lmstep).  w_only: the step in w with
    tau held (the initialisation of the paper's remark rem:solver), i.e. the
    least-squares problem in the columns of J~_w alone; dtau = 0."""
    m = jac["H"].shape[0] - n
    if w_only:
        if solver == "qr":
            dw = np.linalg.lstsq(jac["Jt"][:, :n], -jac["Ft"], rcond=None)[0]
        else:
            L = np.linalg.cholesky(jac["H"][:n, :n])
            dw = np.linalg.solve(L.T, np.linalg.solve(L, -jac["g"][:n]))
        return np.r_[dw, np.zeros(m)]
    if solver == "qr":
        A = np.vstack([jac["Jt"], np.hstack([np.zeros((m, n)), np.sqrt(lam) * np.eye(m)])])
        b = -np.r_[jac["Ft"], np.zeros(m)]
        return np.linalg.lstsq(A, b, rcond=None)[0]
    Hl = jac["H"].copy()
    Hl[n:, n:] += lam * np.eye(m)
    L = np.linalg.cholesky(Hl)
    y = np.linalg.solve(L, -jac["g"])
    return np.linalg.solve(L.T, y)


def gn_step(rom: ROM, mu, w, tau, lam=0.0, c1=1e-4, max_backtrack=30, tol=1e-8, solver="normal", w_only=False):
    """One step from z_n = (w, tau).  Returns (w_new, tau_new, info).

    info: J_old, J_new, alpha, norm_S, norm_T (at z_n), n_backtrack,
    converged (z_n already meets the tolerance; no step taken), status
    ("ok", "converged", "linesearch", "singular", "invalid").  w_only: a step
    in w with tau held, converged when |S~| <= tol."""
    n = rom.n
    jac = rom.jacobian(mu, w, tau)
    g = jac["g"]
    info = {"J_old": jac["J"], "J_new": jac["J"], "alpha": 0.0, "norm_S": float(np.linalg.norm(g[:n])),
            "norm_T": float(np.linalg.norm(g[n:])), "n_backtrack": 0, "converged": False, "status": "ok"}
    if not np.isfinite(jac["J"]):
        info["status"] = "invalid"
        return w, tau, info
    if info["norm_S"] <= tol and (w_only or info["norm_T"] <= tol):
        info["converged"] = True
        info["status"] = "converged"
        return w, tau, info
    try:
        dz = lm_direction(jac, n, lam, solver, w_only)
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


def adapt_lambda(lam, alpha):
    """Reading of the adaptive regularisation (the paper cites a rule it does
    not state): lambda / 10 after a step accepted at alpha = 1 (0 below
    1e-12), max(10 lambda, 1e-8) after a step accepted at alpha < 1."""
    if alpha == 1.0:
        return 0.0 if lam * 0.1 < 1e-12 else lam * 0.1
    return max(10.0 * lam, 1e-8)


def lm_solve(rom: ROM, mu, w0, tau0, lam=0.0, tol=1e-8, max_it=50, presolve=False, adaptive=False,
             c1=1e-4, max_backtrack=30):
    """The whole iteration from (w0, tau0), with the options of the paper.

    presolve: the initialisation of remark rem:solver, w0 = argmin_w
    |R~(w, tau0)|, computed by steps in w with tau held until |S~| <= tol (a
    failed line search ends it early); then full steps from that iterate.
    adaptive: lambda updated by adapt_lambda after every accepted step.
    Every step (in w or full) counts towards max_it.  Returns (w, tau, info)
    with status "converged", "max_it", "linesearch", "singular" or
    "invalid", the step count and the w-step count."""
    n = rom.n
    w, tau = np.array(w0, dtype=float), np.array(tau0, dtype=float)
    it = it_w = 0
    wonly = presolve
    while True:
        jac = rom.jacobian(mu, w, tau)
        if not np.isfinite(jac["J"]):
            return w, tau, {"status": "invalid", "iterations": it, "w_iterations": it_w}
        g = jac["g"]
        nS, nT = np.linalg.norm(g[:n]), np.linalg.norm(g[n:])
        if wonly and nS <= tol:
            wonly = False
        if not wonly and nS <= tol and nT <= tol:
            return w, tau, {"status": "converged", "iterations": it, "w_iterations": it_w}
        if it >= max_it:
            return w, tau, {"status": "max_it", "iterations": it, "w_iterations": it_w}
        try:
            dz = lm_direction(jac, n, lam, "normal", wonly)
        except np.linalg.LinAlgError:
            return w, tau, {"status": "singular", "iterations": it, "w_iterations": it_w}
        it += 1
        it_w += int(wonly)
        slope = float(g @ dz)
        alpha, accepted = 1.0, False
        for bt in range(max_backtrack + 1):
            wt, tt = w + alpha * dz[:n], tau + alpha * dz[n:]
            if rom.residual(mu, wt, tt)["J"] <= jac["J"] + c1 * alpha * slope:
                accepted = True
                break
            alpha *= 0.5
        if accepted:
            w, tau = wt, tt
            if adaptive:
                lam = adapt_lambda(lam, alpha)
        elif wonly:
            wonly = False
        else:
            return w, tau, {"status": "linesearch", "iterations": it, "w_iterations": it_w}
