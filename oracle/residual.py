"""Element residual R_e, distortion N_e and their Jacobians (oracle; test infrastructure).

Follows Section 2 of the paper:

* the conservation law is posed on the reference domain through the mapping
  G (eq. (claw-ref)) with the transformed flux F = g f(U) G^{-T} of
  eq. (p2r-flux), G = grad_0 G, g = det G;
* the discretisation has the assembled form R = sum_e P_e R_e(U_e, U_e', x_e)
  of eq. (hdm_elem) with element DoFs U_e, neighbour DoFs U_e' and element
  mapping DoFs x_e;
* the distortion residual N_e = kappa (eta_e(x_e) - eta_e(X_e)) uses the
  element distortion eta_e of eq. (dist_elem1) with exponent 2/d = 1.

The DG weak form (a reading; the paper only says "standard nodal DG"):
    R_e[i] = sum_faces int phi_i H(U-, U+, n~) dS - int grad_0 phi_i : F dX
             - int phi_i S dX,
with the transformed source S = g s of eq. (p2r-flux) (the source of the
space-time Burgers problem, eq. (burgers), at the mapped point; else 0).
The surface term is written with Nanson's relation,
n~ = g G^{-T} N dS_0 per unit edge parameter, evaluated here literally.
Jacobians come from forward-mode dual numbers (``oracle.dual``).

Everything is evaluated literally from G, g and the reference Jacobian J0;
nothing is simplified, so that ``oracle.physdg`` (plain DG on the physical
mesh) is an independent check of the transformation.
"""
from __future__ import annotations

import numpy as np

from . import physics as ph
from . import refelem as re
from .dual import Dual, ein, lift, maximum, stack, where


def params_of(wl) -> dict:
    return {"pde": wl.pde, "p": wl.p, "n_c": wl.n_c, "gamma": wl.gamma, "kappa": wl.kappa,
            "eps_g": wl.eps_g, "bc_mu_scale": wl.bc_mu_scale, "all_farfield": wl.all_farfield,
            "src_amp": getattr(wl, "src_amp", 0.0), "bc_spacetime": getattr(wl, "bc_spacetime", False)}


# ------------------------------------------------------------ gather maps
def gather_maps(mesh, p: int, n_c: int):
    """Index maps of the assembly operators (Section 2.3):
    U_e = U[P_e], U_e' = U[P_n] (-1 marks a boundary face slot, value 0),
    x_e = x[Q_e].  U_e' holds, for each face f of e and each node k of that
    face ordered by e's edge parameter, the neighbour's DoFs at that node."""
    nn = (p + 1) * (p + 2) // 2
    Ne = mesh.n_elem
    nue = nn * n_c
    P_e = (np.arange(Ne)[:, None] * nue + np.arange(nue)[None, :]).astype(np.int64)
    P_n = -np.ones((Ne, 3, p + 1, n_c), dtype=np.int64)
    for e in range(Ne):
        for f in range(3):
            E = mesh.elem_nbr[e, f]
            if E < 0:
                continue
            g = int(np.nonzero(mesh.elem_nbr[E] == e)[0][0])
            enodes = re.edge_nodes(p, g)
            for k in range(p + 1):
                node = enodes[p - k]        # the neighbour runs the edge the other way
                P_n[e, f, k, :] = (E * nn + node) * n_c + np.arange(n_c)
    Q_e = np.stack([2 * mesh.elem_gnodes, 2 * mesh.elem_gnodes + 1], axis=-1).reshape(Ne, -1).astype(np.int64)
    return P_e, P_n.reshape(Ne, -1), Q_e


def take(a: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """a[idx] with 0 where idx < 0."""
    out = a[np.maximum(idx, 0)]
    return np.where(idx >= 0, out, 0.0)


# ------------------------------------------------------------- geometry
def _jac(xn, dphi):
    """J[e, q, a, b] = sum_n x_n[a] d phi_n / d xi_b."""
    return ein("enk,qnl->eqkl", xn, dphi)


def _inv2(J):
    det = J[..., 0, 0] * J[..., 1, 1] - J[..., 0, 1] * J[..., 1, 0]
    row0 = stack([J[..., 1, 1] / det, -1.0 * J[..., 0, 1] / det], axis=-1)
    row1 = stack([-1.0 * J[..., 1, 0] / det, J[..., 0, 0] / det], axis=-1)
    return stack([row0, row1], axis=-2), det


def _mapping(x_e, X_e, dphi):
    """G = J J0^{-1} (the mapping Jacobian of eq. (p2r-stvc)), g = det G, G^{-1}."""
    J = _jac(x_e, dphi)
    J0 = np.einsum("enk,qnl->eqkl", X_e, dphi)
    J0inv = np.linalg.inv(J0)
    detJ0 = np.linalg.det(J0)
    G = ein("eqab,eqbc->eqac", J, J0inv)
    Ginv, g = _inv2(G)
    return G, g, Ginv, J0, J0inv, detJ0


# -------------------------------------------------------------- residual
def element_residual(prm, U_e, x_e, X_e, nbr_e, mu, trace_plus):
    """R_e [E, nn, n_c], N_e [E] (Duals), bad-geometry and non-physical flags [E].

    U_e: Dual [E, nn, n_c]; x_e: Dual [E, nn, 2]; X_e: [E, nn, 2];
    nbr_e: [E, 3] neighbour (>= 0) or -tag; trace_plus(f, s) -> Dual [E, S, n_c]
    gives the neighbour state at the edge parameters s of face f.
    """
    pde, p = prm["pde"], prm["p"]
    nd = U_e.nd
    x_e = lift(x_e, nd)
    xq, wq = re.volume_rule(p)
    phi, dphi = re.basis(p, xq)
    # --- volume term: - int grad_0 phi_i : F dX, F = g f G^{-T}
    G, g, Ginv, J0, J0inv, detJ0 = _mapping(x_e, X_e, dphi)
    uq = ein("qn,enc->eqc", phi, U_e)
    f = ph.flux(pde, uq, prm)                                    # [E, Q, nc, 2]
    F = ein("eqca,eqba->eqcb", f, Ginv) * g[..., None, None]     # g f G^{-T}
    grad0 = np.einsum("eqba,qnb->eqna", J0inv, dphi)             # J0^{-T} grad_xi phi
    vol = ein("eqcb,eqnb->eqnc", F, grad0)
    R = -1.0 * ein("eqnc,eq->enc", vol, wq[None, :] * detJ0)
    if pde == "burgers" and prm.get("src_amp", 0.0) != 0.0:
        # source of eq. (burgers) on the reference domain: S = g s(x(X)),
        # at the mapped physical position x = sum_n x_n phi_n
        xq_phys = ein("qn,ena->eqa", phi, x_e)
        src = ph.burgers_source(xq_phys[..., 0], mu, prm["src_amp"]) * g
        R = R - ein("qn,eq->en", phi, src * (wq[None, :] * detJ0))[..., None]
    bad = (g.v <= prm["eps_g"]).any(axis=1)
    nonphys = np.zeros(U_e.shape[0], dtype=bool)
    if pde == "euler":
        nonphys |= _nonphysical(uq, prm["gamma"])
    # --- surface term: sum_f int phi_i H(U-, U+, n~) ds
    s, ws = re.face_rule(p)
    for fi in range(3):
        pts = re.face_points(fi, s)
        phf, dphf = re.basis(p, pts)
        Gf, gf, Ginvf, J0f, _, _ = _mapping(x_e, X_e, dphf)
        tau_xi = re.VERTS[(fi + 1) % 3] - re.VERTS[fi]
        dXds = np.einsum("esab,b->esa", J0f, tau_xi)
        Nsc = np.stack([dXds[..., 1], -dXds[..., 0]], axis=-1)   # N dS_0 per ds
        nt = ein("esba,esb->esa", Ginvf, Nsc) * gf[..., None]     # g G^{-T} N dS_0
        um = ein("sn,enc->esc", phf, U_e)
        up_int = trace_plus(fi, s)
        up = up_int
        nb = nbr_e[:, fi]
        for tag in (1, 2, 3, 4):
            sel = nb == -tag
            if sel.any():
                ub = ph.boundary_state(pde, tag, um, nt, mu, prm)
                up = where(sel[:, None, None], ub, up)
        H = ph.numerical_flux(pde, um, up, nt, prm)               # [E, S, nc]
        R = R + ein("sn,esc->enc", phf * ws[:, None], H)
        if pde == "euler":
            nonphys |= _nonphysical(um, prm["gamma"]) | _nonphysical(up, prm["gamma"])
    # --- distortion, eq. (dist_elem1) with 2/d = 1
    eta = _eta(G, g, detJ0, wq, prm["eps_g"])
    G0 = np.einsum("eqab,eqbc->eqac", J0, J0inv)
    g0 = np.linalg.det(G0)
    eta0 = _eta(Dual.const(G0, nd), Dual.const(g0, nd), detJ0, wq, prm["eps_g"])
    N = prm["kappa"] * (eta - eta0)
    return R, N, bad, nonphys


def _eta(G, g, detJ0, wq, eps):
    nG2 = (G * G).sum(axis=-1).sum(axis=-1)
    m = maximum(g, Dual.const(np.full(g.shape, eps), g.nd))
    r = nG2 / m
    return ein("eq,eq->e", r * r, wq[None, :] * detJ0)


def _nonphysical(u: Dual, gamma: float) -> np.ndarray:
    rho = u.v[..., 0]
    E = u.v[..., 3]
    with np.errstate(divide="ignore", invalid="ignore"):
        p = (gamma - 1.0) * (E - 0.5 * (u.v[..., 1] ** 2 + u.v[..., 2] ** 2) / rho)
    bad = (rho <= 0.0) | ~(p > 0.0)
    return bad.reshape(bad.shape[0], -1).any(axis=1)


def trace_from_gathered(p: int, Un: Dual):
    """Neighbour trace from U_e' [E, 3, p+1, nc] by the 1-D Lagrange basis on the edge."""
    def tp(fi, s):
        L = re.lagrange_1d(p, s)
        return ein("sk,ekc->esc", L, Un[:, fi])
    return tp


# --------------------------------------------------------- per-element API
class Problem:
    """Mesh + discretisation data of one workload (oracle side)."""

    def __init__(self, wl):
        self.wl = wl
        self.prm = params_of(wl)
        self.p = wl.p
        self.nc = wl.n_c
        self.nn = wl.n_nodes
        self.nue = self.nn * self.nc
        self.nun = 3 * (self.p + 1) * self.nc
        self.nxe = 2 * self.nn
        self.P_e, self.P_n, self.Q_e = gather_maps(wl.mesh, wl.p, wl.n_c)
        self.X = wl.X
        self.nbr = wl.mesh.elem_nbr

    def evaluate(self, elems, Ue, Une, xe, mu, jac: bool):
        """Element residuals at gathered values Ue [E, nue], Une [E, nun], xe [E, nxe].

        Returns R [E, nue], N [E], and (if jac) dR/dU_e [E, nue, nue],
        dR/dU_e' [E, nue, nun], dR/dx_e [E, nue, nxe], dN/dx_e [E, nxe],
        plus bad / nonphys flags."""
        E = len(elems)
        nd = (self.nue + self.nun + self.nxe) if jac else 0
        Xe = take(self.X, self.Q_e[elems]).reshape(E, self.nn, 2)
        if jac:
            U = Dual.seed(Ue, 0, nd)
            Un = Dual.seed(Une, self.nue, nd)
            x = Dual.seed(xe, self.nue + self.nun, nd)
        else:
            U, Un, x = Dual.const(Ue, 0), Dual.const(Une, 0), Dual.const(xe, 0)
        U = Dual(U.v.reshape(E, self.nn, self.nc), U.d.reshape(E, self.nn, self.nc, nd))
        Un = Dual(Un.v.reshape(E, 3, self.p + 1, self.nc), Un.d.reshape(E, 3, self.p + 1, self.nc, nd))
        x = Dual(x.v.reshape(E, self.nn, 2), x.d.reshape(E, self.nn, 2, nd))
        R, N, bad, nonphys = element_residual(self.prm, U, x, Xe, self.nbr[elems], mu,
                                              trace_from_gathered(self.p, Un))
        Rv = R.v.reshape(E, self.nue)
        out = {"R": Rv, "N": N.v, "bad": bad, "nonphys": nonphys}
        if jac:
            Rd = R.d.reshape(E, self.nue, nd)
            out["dRdU"] = Rd[:, :, :self.nue]
            out["dRdUn"] = Rd[:, :, self.nue:self.nue + self.nun]
            out["dRdx"] = Rd[:, :, self.nue + self.nun:]
            out["dNdx"] = N.d[:, self.nue + self.nun:]
        return out

    def gather_state(self, elems, U, x):
        return U[self.P_e[elems]], take(U, self.P_n[elems]), x[self.Q_e[elems]]


def hdm_assemble(prob: Problem, mu, U, x, jac: bool = True, chunk: int = 1024):
    """Full-order assembly over all N_e elements (eq. (hdm_elem)): the global
    residual R [N_u] (DG blocks are disjoint, P_e^T P_E = delta_eE I), N [N_e]
    and, if jac, the element Jacobian blocks of eq. (hdm_elem_jac1)."""
    Ne = prob.wl.mesh.n_elem
    R = np.zeros(prob.wl.N_u)
    out = {"N": np.zeros(Ne), "n_bad": 0}
    if jac:
        out.update(dRdU=np.zeros((Ne, prob.nue, prob.nue)), dRdUn=np.zeros((Ne, prob.nue, prob.nun)),
                   dRdx=np.zeros((Ne, prob.nue, prob.nxe)), dNdx=np.zeros((Ne, prob.nxe)))
    for a in range(0, Ne, chunk):
        el = np.arange(a, min(Ne, a + chunk))
        Ue, Une, xe = prob.gather_state(el, U, x)
        r = prob.evaluate(el, Ue, Une, xe, mu, jac)
        R[prob.P_e[el]] = r["R"]
        out["N"][el] = r["N"]
        out["n_bad"] += int((r["bad"] | r["nonphys"]).sum())
        if jac:
            for k in ("dRdU", "dRdUn", "dRdx", "dNdx"):
                out[k][el] = r[k]
    out["R"] = R
    return out
