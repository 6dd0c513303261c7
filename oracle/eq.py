"""Element-wise EQ hyperreduced assembly (oracle; test infrastructure).

Section 3.1 and Appendix A of the paper.  For an EQ set {(e_k, rho_k)}:

* gathers (at ROM creation): Phi_e = P_e^T Phi, Phi_e' = P_e'^T Phi,
  Psi_e = Q_e^T Psi, X_e = Q_e^T X (end of Section 3.0, eq. (ift-res-elem2));
* lift: U_e = Phi_e w, U_e' = Phi_e' w, x_e = X_e + Psi_e tau;
* objective, eq. (ift-opt-eqp2): J~ = sum_k rho_k/2 (|R_e|^2 + N_e^2);
* gradient (the hyperreduced residuals S~, T~ of eq. (ift-eqp-res0)):
  S~ = sum rho (Phi_e^T dR/dU_e^T + Phi_e'^T dR/dU_e'^T) R_e,
  T~ = sum rho Psi_e^T (dR/dx_e^T R_e + dN/dx_e^T N_e);
* Gauss-Newton matrix, eq. (levmarq-elem):
  H = sum rho [A_e B_e]^T [A_e B_e] + rho [0 a_e]^T [0 a_e] with
  A_e = dR/dU_e Phi_e + dR/dU_e' Phi_e', B_e = dR/dx_e Psi_e, a_e = dN/dx_e Psi_e;
* the stacked least-squares rows F~ = [sqrt(rho_k) R_e ; sqrt(rho_k) N_e] and
  J~_z = [sqrt(rho_k) [A_e B_e] ; sqrt(rho_k) [0 a_e]] (eq. (ift-eqp-res)),
  element rows first (k-major), then the n_s distortion rows.
An evaluation point where any sampled element has g <= eps or a
non-physical state (Euler: rho <= 0 or p <= 0 at a flux point) has J~ = +inf.
"""
from __future__ import annotations

import numpy as np

from .residual import Problem, take


class ROM:
    def __init__(self, prob: Problem, Phi, Psi, eq_elem, eq_rho):
        self.prob = prob
        self.Phi, self.Psi = Phi, Psi
        self.eq_elem = np.asarray(eq_elem, dtype=np.int64)
        self.eq_rho = np.asarray(eq_rho, dtype=np.float64)
        self.n, self.m = Phi.shape[1], Psi.shape[1]
        el = self.eq_elem
        self.Phi_s = Phi[prob.P_e[el]]                                  # [n_s, nue, n]
        Pn = prob.P_n[el]
        self.Phin_s = np.where((Pn >= 0)[..., None], Phi[np.maximum(Pn, 0)], 0.0)
        self.Psi_s = Psi[prob.Q_e[el]]                                  # [n_s, nxe, m]
        self.X_s = take(prob.X, prob.Q_e[el])                           # [n_s, nxe]

    @property
    def n_s(self):
        return self.eq_elem.shape[0]

    def lift(self, w, tau):
        Ue = self.Phi_s @ w
        Une = self.Phin_s @ w
        xe = self.X_s + self.Psi_s @ tau
        return Ue, Une, xe

    def residual(self, mu, w, tau):
        Ue, Une, xe = self.lift(w, tau)
        r = self.prob.evaluate(self.eq_elem, Ue, Une, xe, mu, jac=False)
        rho = self.eq_rho
        invalid = bool((r["bad"] | r["nonphys"]).any())
        J = 0.5 * np.sum(rho * ((r["R"] ** 2).sum(axis=1) + r["N"] ** 2))
        sq = np.sqrt(rho)
        Ft = np.r_[(sq[:, None] * r["R"]).ravel(), sq * r["N"]]
        PhiT_r = np.einsum("k,krn,kr->n", rho, self.Phi_s, r["R"])
        return {"J": np.inf if invalid else J, "J_raw": J, "Ft": Ft, "PhiT_r": PhiT_r,
                "invalid": invalid, "n_bad": int((r["bad"] | r["nonphys"]).sum()), "elem": r}

    def jacobian(self, mu, w, tau):
        Ue, Une, xe = self.lift(w, tau)
        r = self.prob.evaluate(self.eq_elem, Ue, Une, xe, mu, jac=True)
        rho = self.eq_rho
        A = r["dRdU"] @ self.Phi_s + r["dRdUn"] @ self.Phin_s           # [n_s, nue, n]
        B = r["dRdx"] @ self.Psi_s                                       # [n_s, nue, m]
        a = np.einsum("kx,kxm->km", r["dNdx"], self.Psi_s)               # [n_s, m]
        AB = np.concatenate([A, B], axis=2)                              # [n_s, nue, n+m]
        a0 = np.concatenate([np.zeros((self.n_s, self.n)), a], axis=1)   # [n_s, n+m]
        R, N = r["R"], r["N"]
        g = np.einsum("k,krz,kr->z", rho, AB, R) + np.einsum("k,kz,k->z", rho, a0, N)
        H = np.einsum("k,kry,krz->yz", rho, AB, AB) + np.einsum("k,ky,kz->yz", rho, a0, a0)
        invalid = bool((r["bad"] | r["nonphys"]).any())
        J = 0.5 * np.sum(rho * ((R ** 2).sum(axis=1) + N ** 2))
        sq = np.sqrt(rho)
        Jt = np.vstack([(sq[:, None, None] * AB).reshape(-1, self.n + self.m), sq[:, None] * a0])
        Ft = np.r_[(sq[:, None] * R).ravel(), sq * N]
        C = np.einsum("krz,kr->kz", AB, R) + a0 * N[:, None]
        return {"J": np.inf if invalid else J, "J_raw": J, "g": g, "H": H, "Jt": Jt, "Ft": Ft,
                "invalid": invalid, "elem": r, "A": A, "B": B, "a": a, "C": C}

    def element_contributions(self, mu, w, tau):
        """The elemental reduced residuals of eq. (ift-eqp-res0), one row per
        sampled element and without the weight: C[k] = [S^(e_k); T^(e_k)],
        so that g = sum_k rho_k C[k]."""
        return self.jacobian(mu, w, tau)["C"]


def plain_start(wl, mu):
    """w0 = Phi^T U_fs(mu), tau0 = 0: the free-stream state projected onto the
    (orthonormal) state basis with the identity mapping.  (The paper's own
    start solves a w-only residual minimisation at tau = 0; see its
    solver remark in Section 3.1.3.)"""
    from . import physics as ph
    if wl.pde == "burgers":
        Ufs = np.full(wl.N_u, ph.burgers_boundary_values(
            mu, {"bc_mu_scale": wl.bc_mu_scale, "bc_spacetime": getattr(wl, "bc_spacetime", False)})[0])
    else:
        Ufs = np.tile(ph.euler_free_stream(mu, wl.gamma), wl.N_u // 4)
    return wl.Phi.T @ Ufs, np.zeros(wl.Psi.shape[1])
