"""Global sparse assembly and the rho-masked global objective (oracle; test infrastructure).

This is the "global" route to the EQ quantities: assemble R, dR/dU, dR/dx,
N and dN/dx over all elements as global (sparse) arrays, then apply the
element weights as a diagonal mask D_rho (rho_e on the DoF rows of element e
and on row e of N, zero elsewhere).  With F~ = [D^{1/2} R; D^{1/2} N] as a
function of z = (w, tau), U = Phi w, x = X + Psi tau (Section 3.1),
    J~(z) = 1/2 |F~|^2                          (eq. (ift-opt-eqp1)),
    g     = J~_z^T F~ = [Phi^T R_U^T D R; Psi^T (R_x^T D R + N_x^T D N)]
    H     = J~_z^T J~_z                          (eq. (lmstep), (levmarq-elem)).
Appendix A shows that these equal the element-wise weighted sums, using
P_e^T P_E = delta_eE I; ``oracle.eq`` computes those sums.  Here the
neighbour traces come from the neighbour's own 2-D basis evaluated at the
matching reference point, independently of the gather map P_e'.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import refelem as re
from .dual import Dual, ein
from .residual import Problem, element_residual, take


def _trace_from_neighbour(prob: Problem, elems, Unb: Dual):
    """Neighbour trace from the neighbours' full DoFs Unb [E, 3, nn, nc]."""
    mesh = prob.wl.mesh
    gidx = np.zeros((len(elems), 3), dtype=np.int64)
    for a, e in enumerate(elems):
        for f in range(3):
            E = mesh.elem_nbr[e, f]
            if E >= 0:
                gidx[a, f] = int(np.nonzero(mesh.elem_nbr[E] == e)[0][0])

    def tp(fi, s):
        out = None
        for g in range(3):
            pts = re.face_points(g, 1.0 - s)
            ph_n, _ = re.basis(prob.p, pts)
            val = ein("sn,enc->esc", ph_n, Unb[:, fi])
            sel = (gidx[:, fi] == g)[:, None, None]
            if out is None:
                out = val * sel
            else:
                out = out + val * sel
        return out
    return tp


def global_assemble(prob: Problem, mu, U, x):
    """R [N_u], R_U (csr [N_u, N_u]), R_x (csr [N_u, N_x]), N [N_e], N_x (csr [N_e, N_x])."""
    wl = prob.wl
    mesh = wl.mesh
    Ne, nn, nc, nue, nxe = mesh.n_elem, prob.nn, prob.nc, prob.nue, prob.nxe
    elems = np.arange(Ne)
    nbr = mesh.elem_nbr
    nb_idx = np.where(nbr >= 0, nbr, 0)
    Unb_v = U.reshape(Ne, nn, nc)[nb_idx] * (nbr >= 0)[:, :, None, None]   # [Ne, 3, nn, nc]
    nd = nue + 3 * nue + nxe
    Ud = Dual.seed(U.reshape(Ne, nue), 0, nd)
    Nbd = Dual.seed(Unb_v.reshape(Ne, 3 * nue), nue, nd)
    xd = Dual.seed(x[prob.Q_e], 4 * nue, nd)
    Ud = Dual(Ud.v.reshape(Ne, nn, nc), Ud.d.reshape(Ne, nn, nc, nd))
    Nbd = Dual(Nbd.v.reshape(Ne, 3, nn, nc), Nbd.d.reshape(Ne, 3, nn, nc, nd))
    xd = Dual(xd.v.reshape(Ne, nn, 2), xd.d.reshape(Ne, nn, 2, nd))
    Xe = take(prob.X, prob.Q_e).reshape(Ne, nn, 2)
    R, N, bad, nonphys = element_residual(prob.prm, Ud, xd, Xe, nbr, mu,
                                          _trace_from_neighbour(prob, elems, Nbd))
    Rv = R.v.reshape(Ne, nue)
    Rd = R.d.reshape(Ne, nue, nd)
    rows, cols, vals = [], [], []
    xr, xc, xv = [], [], []
    for e in range(Ne):
        re_rows = prob.P_e[e]
        rows.append(np.repeat(re_rows, nue))
        cols.append(np.tile(prob.P_e[e], nue))
        vals.append(Rd[e, :, :nue].ravel())
        for f in range(3):
            E = nbr[e, f]
            if E < 0:
                continue
            blk = Rd[e, :, nue + f * nue: nue + (f + 1) * nue]
            rows.append(np.repeat(re_rows, nue))
            cols.append(np.tile(prob.P_e[E], nue))
            vals.append(blk.ravel())
        xr.append(np.repeat(re_rows, nxe))
        xc.append(np.tile(prob.Q_e[e], nue))
        xv.append(Rd[e, :, 4 * nue:].ravel())
    N_u, N_x = wl.N_u, prob.X.shape[0]
    RU = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N_u, N_u))
    Rx = sp.csr_matrix((np.concatenate(xv), (np.concatenate(xr), np.concatenate(xc))), shape=(N_u, N_x))
    Nx = sp.csr_matrix((N.d[:, 4 * nue:].ravel(),
                        (np.repeat(np.arange(Ne), nxe), prob.Q_e.ravel())), shape=(Ne, N_x))
    Rg = np.zeros(N_u)
    Rg[prob.P_e] = Rv
    return {"R": Rg, "RU": RU, "Rx": Rx, "N": N.v, "Nx": Nx, "bad": bad, "nonphys": nonphys}


def global_eq(prob: Problem, mu, w, tau, eq_elem, eq_rho):
    """J~, g = [S~; T~], H and Phi^T D R from the global matrices and the D_rho mask."""
    wl = prob.wl
    Phi, Psi = wl.Phi, wl.Psi
    U = Phi @ w
    x = prob.X + Psi @ tau
    A = global_assemble(prob, mu, U, x)
    rho_e = np.zeros(wl.mesh.n_elem)
    np.add.at(rho_e, eq_elem, eq_rho)
    dR = np.repeat(rho_e, prob.nue)
    R, N = A["R"], A["N"]
    RUPhi = A["RU"] @ Phi
    RxPsi = A["Rx"] @ Psi
    NxPsi = A["Nx"] @ Psi
    J = 0.5 * (R @ (dR * R) + N @ (rho_e * N))
    S = RUPhi.T @ (dR * R)
    T = RxPsi.T @ (dR * R) + NxPsi.T @ (rho_e * N)
    Jw = np.hstack([RUPhi, RxPsi]) * np.sqrt(dR)[:, None]
    Jn = np.hstack([np.zeros((NxPsi.shape[0], Phi.shape[1])), NxPsi]) * np.sqrt(rho_e)[:, None]
    H = Jw.T @ Jw + Jn.T @ Jn
    return {"J": J, "g": np.r_[S, T], "H": H, "PhiT_r": Phi.T @ (dR * R), "assembled": A}
