"""Snapshot alignment and mapping-basis update of the greedy loop, Section 3.3.

At a new training parameter the mapping that aligns the solution's features
with those already in the bases solves eq. (align0),
    (w~, x*) = argmin over (w, x) in R^j x R^{N_x} of 1/2 |F(Phi_j w, x; mu)|^2,
F = [R; N] the full-order residual of eq. (ift-obj); the mapping basis then
takes x* - X by Gram-Schmidt, eq. (greedy1).  (The state basis takes the HDM
solution at (x*, mu), which needs a full-order solver: not built.)

Each Gauss-Newton step evaluates F and every element Jacobian block on the
device (hdm_assemble), assembles the global sparse Jacobian
    [R_U Phi_j  R_x; 0  N_x]
on the host from those blocks and the library's own DoF maps, and solves the
damped least-squares problem
    min |J d + F|^2 + lambda |d_x|^2      (lambda > 0 on the node block)
by its sparse normal equations (SuperLU).  The trial points of the Armijo
backtracking (c1 = 1e-4, alpha halved from 1, at most 30 halvings; +inf at
invalid points) are evaluated on the device too.  The sparse solve is the
host part of this offline step, as the program of the weight training is.
"""
from __future__ import annotations

import numpy as np

from . import ift


class Alignment:
    """Alignment problem of eq. (align0) on `prob` with the state basis Phi_j
    (host [N_u, j]); device buffers for one full-order evaluation."""

    def __init__(self, prob: ift.Problem, Phi_j):
        import torch
        self.prob = prob
        self.Phi = np.ascontiguousarray(Phi_j, dtype=np.float64)
        if self.Phi.ndim != 2 or self.Phi.shape[0] != prob.N_u:
            raise ValueError(f"Phi_j must be [{prob.N_u}, j]")
        self.j = self.Phi.shape[1]
        Ne, nue, nun, nxe = prob.n_elem, prob.nue, prob.nun, prob.nxe
        self.Pe = np.arange(Ne)[:, None] * nue + np.arange(nue)[None, :]
        self.Pn = prob.neighbour_map()
        gn = prob._gn.astype(np.int64)
        self.Qe = np.stack([2 * gn, 2 * gn + 1], axis=-1).reshape(Ne, nxe)
        dev = torch.device("cuda:0")
        z = lambda k: torch.zeros(k, dtype=torch.float64, device=dev)
        self.dev = dev
        self.buf = dict(R=z(prob.N_u), N=z(Ne), dRdU=z(Ne * nue * nue), dRdUn=z(Ne * nue * nun),
                        dRdx=z(Ne * nue * nxe), dNdx=z(Ne * nxe),
                        n_bad=torch.zeros(1, dtype=torch.int32, device=dev))

    def _evaluate(self, mu, w, x, jac: bool):
        import torch
        b = self.buf
        U = torch.tensor(self.Phi @ np.asarray(w, dtype=np.float64), device=self.dev)
        xt = torch.tensor(np.asarray(x, dtype=np.float64), device=self.dev)
        keys = ("R", "N", "dRdU", "dRdUn", "dRdx", "dNdx", "n_bad") if jac else ("R", "N", "n_bad")
        self.prob.hdm_assemble(mu, U, xt, **{k: b[k] for k in keys})
        torch.cuda.synchronize()
        return {k: b[k].cpu().numpy() for k in keys}

    def objective(self, mu, w, x) -> float:
        """1/2 |F|^2 at (w, x); +inf at an invalid point."""
        o = self._evaluate(mu, w, x, jac=False)
        if int(o["n_bad"][0]) > 0:
            return np.inf
        return 0.5 * (float(o["R"] @ o["R"]) + float(o["N"] @ o["N"]))

    def jacobian(self, mu, w, x):
        """F, the sparse dF/d(w, x) and the invalid-element count at (w, x)."""
        import scipy.sparse as sp
        p = self.prob
        Ne, nue, nun, nxe = p.n_elem, p.nue, p.nun, p.nxe
        o = self._evaluate(mu, w, x, jac=True)
        dU = o["dRdU"].reshape(Ne, nue, nue)
        dUn = o["dRdUn"].reshape(Ne, nue, nun)
        dx = o["dRdx"].reshape(Ne, nue, nxe)
        dN = o["dNdx"].reshape(Ne, nxe)
        # R_U Phi_j element by element: own DoFs, then the neighbour traces
        Phin = np.where(self.Pn[..., None] >= 0, self.Phi[np.maximum(self.Pn, 0)], 0.0)   # [Ne, nun, j]
        RUPhi = (np.einsum("erc,ecj->erj", dU, self.Phi[self.Pe]) + np.einsum("erc,ecj->erj", dUn, Phin))
        RUPhi = RUPhi.reshape(p.N_u, self.j)
        rows = np.broadcast_to(self.Pe[:, :, None], (Ne, nue, nxe)).ravel()
        cols = np.broadcast_to(self.Qe[:, None, :], (Ne, nue, nxe)).ravel()
        Rx = sp.csr_matrix((dx.ravel(), (rows, cols)), shape=(p.N_u, p.N_x))
        nrows = np.broadcast_to(np.arange(Ne)[:, None], (Ne, nxe)).ravel()
        Nx = sp.csr_matrix((dN.ravel(), (nrows, self.Qe.ravel())), shape=(Ne, p.N_x))
        F = np.r_[o["R"], o["N"]]
        Jw = np.vstack([RUPhi, np.zeros((Ne, self.j))])
        Jx = sp.vstack([Rx, Nx]).tocsr()
        return F, Jw, Jx, int(o["n_bad"][0])

    def direction(self, mu, w, x, lam: float):
        """The damped least-squares step (dw, dx) and {F, J, g} at (w, x)
        (a zero step and J = +inf at an invalid point), from the sparse
        normal equations
            [Jw^T Jw  Jw^T Jx; Jx^T Jw  Jx^T Jx + lambda I] d = -[Jw^T F; Jx^T F]."""
        import scipy.sparse as sp
        import scipy.sparse.linalg as spl
        if not lam > 0.0:
            raise ValueError("lambda must be positive (rigid translations of the nodes are null directions)")
        F, Jw, Jx, n_bad = self.jacobian(mu, w, x)
        Nx = Jx.shape[1]
        if n_bad:   # invalid point: no step
            return np.zeros(self.j), np.zeros(Nx), {"F": F, "J": np.inf, "g": np.full(self.j + Nx, np.nan)}
        g = np.r_[Jw.T @ F, Jx.T @ F]
        J = 0.5 * float(F @ F)
        A = sp.bmat([[sp.csr_matrix(Jw.T @ Jw), sp.csr_matrix(Jx.T @ Jw).T],
                     [sp.csr_matrix(Jx.T @ Jw), (Jx.T @ Jx + lam * sp.identity(Nx)).tocsr()]]).tocsc()
        d = spl.spsolve(A, -g)
        return d[:self.j], d[self.j:], {"F": F, "J": J, "g": g}

    def step(self, mu, w, x, lam: float, c1: float = 1e-4, max_backtrack: int = 30):
        """One Gauss-Newton step with Armijo backtracking.  Returns (w, x,
        info) with J_old, J_new, alpha, n_backtrack, norm_g and status
        ("ok", "linesearch", "invalid")."""
        w = np.asarray(w, dtype=np.float64)
        x = np.asarray(x, dtype=np.float64)
        dw, dx, d = self.direction(mu, w, x, lam)
        info = {"J_old": d["J"], "J_new": d["J"], "alpha": 0.0, "n_backtrack": 0,
                "norm_g": float(np.linalg.norm(d["g"])), "status": "ok"}
        if not np.isfinite(d["J"]):
            info["status"] = "invalid"
            info["norm_g"] = np.inf
            return w, x, info
        slope = float(d["g"] @ np.r_[dw, dx])
        alpha = 1.0
        for bt in range(max_backtrack + 1):
            wt, xt = w + alpha * dw, x + alpha * dx
            Jt = self.objective(mu, wt, xt)
            if Jt <= d["J"] + c1 * alpha * slope:
                info.update(J_new=Jt, alpha=alpha, n_backtrack=bt)
                return wt, xt, info
            alpha *= 0.5
        info["status"] = "linesearch"
        info["n_backtrack"] = max_backtrack + 1
        return w, x, info


def gram_schmidt_append(B, v):
    """[B q], q the component of v orthogonal to the orthonormal columns of
    B (two passes of classical Gram-Schmidt), normalised: eq. (greedy1)."""
    B = np.asarray(B, dtype=np.float64)
    q = np.array(v, dtype=np.float64)
    for _ in range(2):
        q -= B @ (B.T @ q)
    nq = np.linalg.norm(q)
    if not nq > 0.0:
        raise ValueError("v lies in the span of B")
    return np.hstack([B, (q / nq)[:, None]])
