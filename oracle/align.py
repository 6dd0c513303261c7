"""Snapshot alignment and basis update of the greedy loop (oracle; test infrastructure).

Section 3.3 of the paper.  At the new training parameter mu_{j+1} the
mapping that aligns the solution's features with those already in the
bases solves eq. (align0),
    (w~, x*) = argmin over (w, x) in R^j x R^{N_x} of 1/2 |F(Phi_j w, x; mu)|^2,
with the full-order residual F(U, x) = [R(U; x, mu); N(x)] of eq.
(ift-obj) and the whole node vector x free.  The mapping basis then takes
x* - X by Gram-Schmidt, eq. (greedy1) (the state basis takes the HDM
solution at (x*, mu_{j+1}), which needs the HDM solver and is not built).

Readings (the paper defers the solver to a cited work): Gauss-Newton on
(w, x) with the least-squares step
    min | [F; 0] + [R_U Phi_j  R_x; 0  N_x; 0  sqrt(lambda) I] Delta |
(the Levenberg-Marquardt term on the x block, as in eq. (levmarq-step);
lambda > 0, since rigid translations of all nodes leave F unchanged when
the problem has no position-dependent source),
Armijo backtracking (c1 = 1e-4, alpha halved from 1, at most 30 halvings)
on 1/2 |F|^2, +inf at invalid points.  Everything here is dense and meant
for small meshes: R_U, R_x and N_x come from the oracle's global sparse
assembly, the step from a dense lstsq.
"""
from __future__ import annotations

import numpy as np

from .assemble import global_assemble
from .residual import Problem


def residual(prob: Problem, Phi_j, mu, w, x):
    """F = [R; N] at U = Phi_j w and x, and whether the point is invalid."""
    A = global_assemble(prob, mu, Phi_j @ w, x)
    return np.r_[A["R"], A["N"]], bool(A["bad"].any() or A["nonphys"].any()), A


def objective(prob: Problem, Phi_j, mu, w, x) -> float:
    F, invalid, _ = residual(prob, Phi_j, mu, w, x)
    return np.inf if invalid else 0.5 * float(F @ F)


def jacobian(prob: Problem, Phi_j, A):
    """dF/d(w, x) = [R_U Phi_j  R_x; 0  N_x] (dense) from a global assembly."""
    RU, Rx, Nx = A["RU"], A["Rx"], A["Nx"]
    top = np.hstack([RU @ Phi_j, Rx.toarray()])
    bottom = np.hstack([np.zeros((Nx.shape[0], Phi_j.shape[1])), Nx.toarray()])
    return np.vstack([top, bottom])


def direction(prob: Problem, Phi_j, mu, w, x, lam=0.0):
    """The least-squares step (Delta w, Delta x), F, 1/2 |F|^2 and the
    gradient J^T F at (w, x)."""
    F, invalid, A = residual(prob, Phi_j, mu, w, x)
    J = jacobian(prob, Phi_j, A)
    j, Nx = Phi_j.shape[1], x.size
    M = np.vstack([J, np.hstack([np.zeros((Nx, j)), np.sqrt(lam) * np.eye(Nx)])]) if lam > 0 else J
    b = -np.r_[F, np.zeros(Nx)] if lam > 0 else -F
    d = np.linalg.lstsq(M, b, rcond=None)[0]
    return d[:j], d[j:], {"F": F, "J": np.inf if invalid else 0.5 * float(F @ F), "g": J.T @ F, "Jac": J}


def step(prob: Problem, Phi_j, mu, w, x, lam=0.0, c1=1e-4, max_backtrack=30):
    """One Gauss-Newton step of eq. (align0) with Armijo backtracking.
    Returns (w_new, x_new, info) with info J_old, J_new, alpha, n_backtrack,
    norm_g and status ("ok", "linesearch", "invalid")."""
    dw, dx, d = direction(prob, Phi_j, mu, w, x, lam)
    info = {"J_old": d["J"], "J_new": d["J"], "alpha": 0.0, "n_backtrack": 0,
            "norm_g": float(np.linalg.norm(d["g"])), "status": "ok"}
    if not np.isfinite(d["J"]):
        info["status"] = "invalid"
        return w, x, info
    slope = float(d["g"] @ np.r_[dw, dx])
    alpha = 1.0
    for bt in range(max_backtrack + 1):
        wt, xt = w + alpha * dw, x + alpha * dx
        Jt = objective(prob, Phi_j, mu, wt, xt)
        if Jt <= d["J"] + c1 * alpha * slope:
            info.update(J_new=Jt, alpha=alpha, n_backtrack=bt)
            return wt, xt, info
        alpha *= 0.5
    info["status"] = "linesearch"
    info["n_backtrack"] = max_backtrack + 1
    return w, x, info


def gram_schmidt_append(B, v):
    """[B q] with q the part of v orthogonal to the orthonormal columns of B,
    normalised (classical Gram-Schmidt, applied twice), eq. (greedy1)."""
    q = np.array(v, dtype=float)
    for _ in range(2):
        q = q - B @ (B.T @ q)
    return np.hstack([B, (q / np.linalg.norm(q))[:, None]])
