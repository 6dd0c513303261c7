"""EQ-weight training, eq. (eqp-lp)-(eqp-con) of Section 3.2: the element
weights rho >= 0 of smallest sum such that the weights integrate the domain
volume to within delta (the dv constraint) and the weighted reduced
residuals stay within delta / |Xi| (max norm) of the full reduced residuals
at every training solution (the sr and dr constraints).

The columns of the program, the elemental reduced residuals [S^(e); T^(e)]
at each training solution, come from the device: ROM.element_contributions
evaluated at the training solutions of the ROM weighted by the guess
rho_check (rho_check = 1 at the paper's first greedy iteration, where the
solution is the ROM-IFT solution; the previous iteration's weights later).
The guess only selects where the contributions are evaluated: the
accuracy constraints always compare against the unweighted sums over all
elements (the hatted S and T of eq. (eqp-con)), so rho = 1 is feasible for
any guess.
The program itself is small and dense (2 + 2 |Xi| (n + m) rows) and is
solved on the host by HiGHS (scipy.optimize.linprog)."""
from __future__ import annotations

import numpy as np


def element_volumes(X, elem_gnodes) -> np.ndarray:
    """|Omega_0,e| of the straight-sided reference elements: X [n_gnode, 2],
    elem_gnodes [n_elem, nn] (vertices first)."""
    X = np.asarray(X, dtype=np.float64).reshape(-1, 2)
    v = X[np.asarray(elem_gnodes)[:, :3]]
    d1, d2 = v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]
    return 0.5 * np.abs(d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0])


def program(contribs, vol, delta: float, delta_vol=None):
    """The linear program min 1^T rho s.t. A_ub rho <= b_ub, rho >= 0.

    contribs: list over the training set Xi of [N_e, n + m] arrays, row e the
    unweighted elemental residuals of element e at that training solution;
    vol: [N_e] element volumes; delta: the accuracy tolerance (each weighted
    residual within delta / |Xi| of the full one, max norm); delta_vol: the
    relative volume tolerance (default delta, as in the paper, which uses
    one tolerance for both).  The full reduced residuals the weighted ones
    must match are the unweighted sums sum_e c_e (eq. (eqp-con)), whatever
    weights the training solutions were computed with.  Each block of rows
    is divided by its largest coefficient (the same constraints, with O(1)
    coefficients for the solver)."""
    vol = np.asarray(vol, dtype=np.float64)
    N = vol.size
    dv = delta if delta_vol is None else delta_vol
    V = float(vol.sum())
    sv = float(vol.max())
    rows = [vol[None, :] / sv, -vol[None, :] / sv]
    rhs = [np.array([(1 + dv) * V / sv]), np.array([(dv - 1) * V / sv])]
    tol = delta / max(1, len(contribs))
    for Cj in contribs:
        Cj = np.asarray(Cj, dtype=np.float64)
        sj = max(float(np.abs(Cj).max()), 1e-300)
        target = Cj.sum(axis=0)
        rows += [Cj.T / sj, -Cj.T / sj]
        rhs += [(target + tol) / sj, (-target + tol) / sj]
    return np.ones(N), np.vstack(rows), np.concatenate(rhs)


def train_weights(contribs, vol, delta: float, delta_vol=None, drop: float = 1e-12, feas_tol: float = 1e-10):
    """Solves the program; returns (rho, info) with rho [N_e] (entries below
    drop * max(rho) set to 0) and info {"status", "message", "nnz",
    "objective", "max_violation"} (the violation of the normalised rows,
    recomputed with the returned rho).  feas_tol is HiGHS's primal
    feasibility tolerance on the normalised rows."""
    from scipy.optimize import linprog
    c, A, b = program(contribs, vol, delta, delta_vol)
    res = linprog(c, A_ub=A, b_ub=b, bounds=(0, None), method="highs",
                  options={"primal_feasibility_tolerance": feas_tol})
    if res.x is None:
        return None, {"status": int(res.status), "message": res.message}
    rho = np.asarray(res.x, dtype=np.float64).copy()
    rho[rho < drop * max(rho.max(), 1e-300)] = 0.0
    viol = float(np.max(A @ rho - b))
    return rho, {"status": int(res.status), "message": res.message, "nnz": int(np.count_nonzero(rho)),
                 "objective": float(rho.sum()), "max_violation": viol}
