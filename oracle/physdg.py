"""Plain DG residual on the physical mesh (oracle; test infrastructure).

The transformed conservation law of eq. (claw-ref)/(p2r-flux) is equivalent
to the physical one of eq. (claw-phys) whenever the mapping is a
diffeomorphism (Section 2.2).  For the discrete residual this means: the
transformed residual on the reference mesh with mapping coefficients x must
equal the ordinary DG residual computed directly on the physical mesh x
(physical basis gradients J^{-T} grad_xi phi, physical measure det J, scaled
physical edge normal).  This routine computes the latter without G, g or the
reference Jacobian, as an independent check of ``oracle.residual``.
Values only; neighbour traces come from the neighbour's own 2-D basis.
"""
from __future__ import annotations

import numpy as np

from . import physics as ph
from . import refelem as re


def physical_residual(wl, mu, U, x):
    p, nc = wl.p, wl.n_c
    nn = wl.n_nodes
    mesh = wl.mesh
    Ne = mesh.n_elem
    prm = {"gamma": wl.gamma, "bc_mu_scale": wl.bc_mu_scale, "all_farfield": wl.all_farfield,
           "bc_spacetime": getattr(wl, "bc_spacetime", False)}
    amp = getattr(wl, "src_amp", 0.0) if wl.pde == "burgers" else 0.0
    Ue = U.reshape(Ne, nn, nc)
    xe = x.reshape(-1, 2)[mesh.elem_gnodes]                      # [Ne, nn, 2]
    xq, wq = re.volume_rule(p)
    phi, dphi = re.basis(p, xq)
    R = np.zeros((Ne, nn, nc))
    for e in range(Ne):
        for q in range(len(wq)):
            J = xe[e].T @ dphi[q]                                 # dx/dxi
            gradx = dphi[q] @ np.linalg.inv(J)                    # [nn, 2] = J^{-T} grad_xi phi
            u = phi[q] @ Ue[e]
            f = ph.flux(wl.pde, u[None], prm).v[0]               # [nc, 2]
            R[e] -= wq[q] * np.linalg.det(J) * gradx @ f.T
            if amp != 0.0:
                # - int phi_i s dx over the physical element, s at the point's x
                xpt = phi[q] @ xe[e]
                R[e, :, 0] -= wq[q] * np.linalg.det(J) * phi[q] * (amp * np.exp(float(mu[1]) * xpt[0]))
        s, ws = re.face_rule(p)
        for fi in range(3):
            pts = re.face_points(fi, s)
            phf, dphf = re.basis(p, pts)
            nb = mesh.elem_nbr[e, fi]
            for k in range(len(s)):
                J = xe[e].T @ dphf[k]
                t = J @ (re.VERTS[(fi + 1) % 3] - re.VERTS[fi])
                nt = np.array([t[1], -t[0]])
                um = phf[k] @ Ue[e]
                if nb >= 0:
                    g = int(np.nonzero(mesh.elem_nbr[nb] == e)[0][0])
                    pn = re.face_points(g, np.array([1.0 - s[k]]))
                    phn, _ = re.basis(p, pn)
                    up = phn[0] @ Ue[nb]
                else:
                    up = ph.boundary_state(wl.pde, -nb, um[None], nt[None], mu, prm).v[0]
                H = ph.numerical_flux(wl.pde, um[None], up[None], nt[None], prm).v[0]
                R[e] += ws[k] * np.outer(phf[k], H)
    return R.reshape(-1)
