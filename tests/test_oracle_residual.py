"""Pins of the oracle's element residual, distortion and Jacobians against
what the paper and the mathematics fix (Section 2, eqs. (claw-ref),
(p2r-flux), (hdm_elem), (dist_elem0)-(dist_elem1), Appendix A)."""
import numpy as np
import pytest

import synth
from conftest import rel
from oracle import physdg, physics as ph, refelem as re
from oracle import residual as rs


def _state_fs(wl, mu):
    if wl.pde == "burgers":
        return np.full(wl.N_u, ph.burgers_inflow(mu, wl.bc_mu_scale))
    return np.tile(ph.euler_free_stream(mu, wl.gamma), wl.N_u // 4)


def test_mesh_invariants(tiny, euler_small):
    for wl, area in ((tiny, 1.0), (euler_small, 2.0)):
        mesh = wl.mesh
        assert mesh.n_elem == 2 * mesh.nx * mesh.ny
        xy = mesh.node_coords()
        a = 0.5 * ((xy[:, 1, 0] - xy[:, 0, 0]) * (xy[:, 2, 1] - xy[:, 0, 1])
                   - (xy[:, 2, 0] - xy[:, 0, 0]) * (xy[:, 1, 1] - xy[:, 0, 1]))
        assert (a > 0).all() and abs(a.sum() - area) < 1e-13
        nb = mesh.elem_nbr
        for e in range(mesh.n_elem):
            for f in range(3):
                E = nb[e, f]
                if E >= 0:
                    assert (nb[E] == e).sum() == 1
                    g = int(np.nonzero(nb[E] == e)[0][0])
                    # shared edge is traversed in opposite directions
                    assert mesh.elem_gnodes[e, f] == mesh.elem_gnodes[E, (g + 1) % 3]
                    assert mesh.elem_gnodes[e, (f + 1) % 3] == mesh.elem_gnodes[E, g]
    assert (tiny.mesh.elem_nbr < 0).sum() == 4 * 8


@pytest.mark.parametrize("case", ["burgers", "euler_walls", "euler_farfield"])
def test_free_stream_preserved_on_mapped_mesh(case, tiny, euler_small):
    import copy
    wl = tiny if case == "burgers" else copy.copy(euler_small)
    if case == "euler_farfield":
        wl.all_farfield = True
    pb = rs.Problem(wl)
    for k in range(3):
        mu = wl.mus[k].copy()
        if case == "euler_farfield":
            mu[1] = 4.0 - 3.0 * k        # any inflow angle
        x = wl.X + wl.Psi @ wl.tau_eval[k]
        U = _state_fs(wl, mu)
        out = rs.hdm_assemble(pb, mu, U, x, jac=False)
        scale = np.abs(ph.flux(wl.pde, U[:wl.n_c][None], rs.params_of(wl)).v).max()
        assert np.abs(out["R"]).max() < 1e-13 * scale


def test_unmapped_reduction(euler_small):
    wl = euler_small
    pb = rs.Problem(wl)
    mu = wl.mus[0]
    U = wl.Phi @ wl.w_eval[0]
    out = rs.hdm_assemble(pb, mu, U, wl.X.copy(), jac=False)
    assert np.abs(out["N"]).max() < 1e-14
    ref = physdg.physical_residual(wl, mu, U, wl.X.copy())
    assert rel(out["R"], ref) < 1e-13


@pytest.mark.parametrize("which", ["tiny", "euler_small", "st_burgers", "st_burgers_p2"])
def test_transformed_equals_physical_dg(which, request):
    wl = request.getfixturevalue(which)
    pb = rs.Problem(wl)
    for k in (0, 5):
        mu = wl.mus[k]
        U = wl.Phi @ wl.w_eval[k]
        x = wl.X + wl.Psi @ wl.tau_eval[k]
        R = rs.hdm_assemble(pb, mu, U, x, jac=False)["R"]
        assert rel(R, physdg.physical_residual(wl, mu, U, x)) < 1e-13


def test_discrete_conservation(euler_small):
    """sum_e sum_i R_e[i, c] equals the boundary flux: interior faces cancel."""
    wl = euler_small
    pb = rs.Problem(wl)
    mu = wl.mus[1]
    U = wl.Phi @ wl.w_eval[1]
    x = wl.X + wl.Psi @ wl.tau_eval[1]
    R = rs.hdm_assemble(pb, mu, U, x, jac=False)["R"].reshape(-1, wl.n_nodes, 4).sum(axis=(0, 1))
    prm = rs.params_of(wl)
    s, ws = re.face_rule(2)
    xe = x.reshape(-1, 2)[wl.mesh.elem_gnodes]
    Ue = U.reshape(-1, 6, 4)
    bsum = np.zeros(4)
    for e in range(wl.mesh.n_elem):
        for f in range(3):
            tag = -wl.mesh.elem_nbr[e, f]
            if tag <= 0:
                continue
            pts = re.face_points(f, s)
            phi, dphi = re.basis(2, pts)
            for k in range(len(s)):
                t = (xe[e].T @ dphi[k]) @ (re.VERTS[(f + 1) % 3] - re.VERTS[f])
                nt = np.array([[t[1], -t[0]]])
                um = (phi[k] @ Ue[e])[None]
                up = ph.boundary_state("euler", tag, um, nt, mu, prm).v
                bsum += ws[k] * ph.euler_roe(um, up, nt, wl.gamma).v[0]
    assert np.abs(R - bsum).max() < 1e-12 * np.abs(bsum).max()


def test_p1_burgers_closed_form(tiny):
    """Continuous linear u = a + b x + c y on straight P1 elements: away from
    inflow faces R_e[i] = int_e phi_i (u u_x + u_y) dx exactly, which is
    b sum_j u_j |T| (1 + delta_ij) / 12 + c |T| / 3."""
    wl = tiny
    pb = rs.Problem(wl)
    a, b, c = 0.7, 0.4, -0.3
    x = wl.X + wl.Psi @ wl.tau_eval[2]
    xy = x.reshape(-1, 2)[wl.mesh.elem_gnodes]
    uval = a + b * xy[..., 0] + c * xy[..., 1]
    R = rs.hdm_assemble(pb, wl.mus[0], uval.reshape(-1), x, jac=False)["R"].reshape(-1, 3)
    area = 0.5 * ((xy[:, 1, 0] - xy[:, 0, 0]) * (xy[:, 2, 1] - xy[:, 0, 1])
                  - (xy[:, 2, 0] - xy[:, 0, 0]) * (xy[:, 1, 1] - xy[:, 0, 1]))
    M = (np.ones((3, 3)) + np.eye(3)) / 12.0
    ref = b * area[:, None] * (uval @ M) + c * area[:, None] / 3.0
    keep = ~np.isin(wl.mesh.elem_nbr, [-1, -3]).any(axis=1)
    assert keep.sum() > 80
    assert np.abs(R[keep] - ref[keep]).max() < 1e-15 * 100


def test_distortion_closed_forms(euler_small):
    """eta_e = int (|G|_F^2 / max(g, eps))^2: zero change under a similarity
    map, and ((2 + s^2)^2 - 4) |Omega_e| kappa under the shear x = X + s Y e_x."""
    wl = euler_small
    pb = rs.Problem(wl)
    U = wl.Phi @ wl.w_eval[0]
    X = wl.X.reshape(-1, 2)
    th = 0.3
    Q = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    xs = (1.7 * X @ Q.T + np.array([0.2, -0.1])).reshape(-1)
    N = rs.hdm_assemble(pb, wl.mus[0], U, xs, jac=False)["N"]
    assert np.abs(N).max() < 1e-14
    s = 0.37
    xsh = X.copy()
    xsh[:, 0] += s * X[:, 1]
    N = rs.hdm_assemble(pb, wl.mus[0], U, xsh.reshape(-1), jac=False)["N"]
    area = 2.0 / wl.mesh.n_elem
    assert np.abs(N - wl.kappa * ((2 + s * s) ** 2 - 4) * area).max() < 1e-14


def test_invalid_geometry_and_state_flagged(euler_small):
    wl = euler_small
    pb = rs.Problem(wl)
    mu = wl.mus[0]
    U = wl.Phi @ wl.w_eval[0]
    out = rs.hdm_assemble(pb, mu, U, wl.X + wl.Psi @ (60.0 * wl.tau_eval[0]), jac=False)
    assert out["n_bad"] > 0
    Ub = U.copy()
    Ub[0::4][:30] = -0.5                      # negative density on a few nodes
    out = rs.hdm_assemble(pb, mu, Ub, wl.X + wl.Psi @ wl.tau_eval[0], jac=False)
    assert out["n_bad"] > 0
    out = rs.hdm_assemble(pb, mu, U, wl.X + wl.Psi @ wl.tau_eval[0], jac=False)
    assert out["n_bad"] == 0


def _fd_blocks(pb, el, Ue, Une, xe, mu):
    r = pb.evaluate(el, Ue, Une, xe, mu, jac=True)
    res = {}
    for name, arr in (("dRdU", Ue), ("dRdUn", Une), ("dRdx", xe)):
        J = np.zeros_like(r[name])
        for j in range(arr.shape[1]):
            h = 1e-6 * max(1.0, np.abs(arr[:, j]).max())
            ap, am = arr.copy(), arr.copy()
            ap[:, j] += h
            am[:, j] -= h
            args = {"dRdU": lambda a: (a, Une, xe), "dRdUn": lambda a: (Ue, a, xe),
                    "dRdx": lambda a: (Ue, Une, a)}[name]
            J[:, :, j] = (pb.evaluate(el, *args(ap), mu, False)["R"]
                          - pb.evaluate(el, *args(am), mu, False)["R"]) / (2 * h)
        res[name] = J
    Jn = np.zeros_like(r["dNdx"])
    for j in range(xe.shape[1]):
        ap, am = xe.copy(), xe.copy()
        ap[:, j] += 1e-6
        am[:, j] -= 1e-6
        Jn[:, j] = (pb.evaluate(el, Ue, Une, ap, mu, False)["N"] - pb.evaluate(el, Ue, Une, am, mu, False)["N"]) / 2e-6
    res["dNdx"] = Jn
    return r, res


@pytest.mark.parametrize("which", ["tiny", "euler_small", "st_burgers", "st_burgers_p2"])
def test_jacobians_match_central_fd(which, request):
    wl = request.getfixturevalue(which)
    pb = rs.Problem(wl)
    el = np.arange(wl.mesh.n_elem)
    mu = wl.mus[1]
    U = wl.Phi @ wl.w_eval[1]
    x = wl.X + wl.Psi @ wl.tau_eval[1]
    r, fd = _fd_blocks(pb, el, *pb.gather_state(el, U, x), mu)
    for k in ("dRdU", "dRdUn", "dRdx", "dNdx"):
        a, b = r[k], fd[k]
        if wl.pde == "burgers" and k == "dRdx":
            # The Lax-Friedrichs speed max(|u- n_x + n_y|, |u+ n_x + n_y|) ties
            # on horizontal inflow faces (n_x = 0); d/dy of their nodes is a
            # one-sided derivative there (tie rule: the u- branch).
            mask = np.ones_like(a, dtype=bool)
            for e in np.nonzero((wl.mesh.elem_nbr == -3).any(axis=1))[0]:
                f = int(np.nonzero(wl.mesh.elem_nbr[e] == -3)[0][0])
                for node in re.edge_nodes(wl.p, f):
                    mask[e, :, 2 * node + 1] = False
            a, b = a[mask], b[mask]
        assert rel(a, b) < 1e-6, k


def _physical_area(wl, x):
    """Area of each physical element from its boundary, 1/2 sum over edges of
    int (x dy - y dx), with the edge x(s) = sum_k L_k(s) x_k of degree p
    (vertices v_f, v_f+1 and, for p = 2, the mid-edge node f) integrated by
    3-point Gauss-Legendre (exact: the integrand has degree 2p - 1)."""
    xe = x.reshape(-1, 2)[wl.mesh.elem_gnodes]
    t, w = np.polynomial.legendre.leggauss(3)
    s, w = 0.5 * (t + 1.0), 0.5 * w
    area = np.zeros(wl.mesh.n_elem)
    for f in range(3):
        a, b = xe[:, f], xe[:, (f + 1) % 3]
        if wl.p == 1:
            pos = a[:, None] * (1 - s)[None, :, None] + b[:, None] * s[None, :, None]
            der = (b - a)[:, None, :] * np.ones_like(s)[None, :, None]
        else:
            c = xe[:, 3 + f]
            L = [(1 - s) * (1 - 2 * s), s * (2 * s - 1), 4 * s * (1 - s)]
            dL = [4 * s - 3, 4 * s - 1, 4 - 8 * s]
            pos = sum(v[:, None] * l[None, :, None] for v, l in zip((a, b, c), L))
            der = sum(v[:, None] * l[None, :, None] for v, l in zip((a, b, c), dL))
        area += 0.5 * ((pos[..., 0] * der[..., 1] - pos[..., 1] * der[..., 0]) * w[None, :]).sum(axis=1)
    return area


@pytest.mark.parametrize("which", ["st_burgers", "st_burgers_p2"])
def test_constant_source_integrates_physical_area(which, request):
    # b = 0: s = s_0 everywhere, and the nodal basis sums to one, so the source
    # part of sum_i R_e[i] is -s_0 |Omega_e| on the mapped (curved) element;
    # the volume rules integrate det J exactly (degree 2(p - 1) <= 2p)
    import dataclasses
    wl = request.getfixturevalue(which)
    off = dataclasses.replace(wl, src_amp=0.0)
    for k in (0, 3):
        mu = np.array([wl.mus[k][0], 0.0])
        U = wl.Phi @ wl.w_eval[k]
        x = wl.X + wl.Psi @ wl.tau_eval[k]
        Rs = rs.hdm_assemble(rs.Problem(wl), mu, U, x, jac=False)["R"]
        R0 = rs.hdm_assemble(rs.Problem(off), mu, U, x, jac=False)["R"]
        per_elem = (Rs - R0).reshape(wl.mesh.n_elem, -1).sum(axis=1)
        assert rel(per_elem, -wl.src_amp * _physical_area(wl, x)) < 1e-13
        assert abs(_physical_area(wl, x).sum() - 5000.0) < 1e-9   # tangential modes keep the domain


def test_source_grows_with_physical_position(st_burgers):
    # s(x) = s_0 exp(b x) at the mapped point: shifting every node right by
    # d multiplies each element's source part by exp(b d) (a rigid translation
    # leaves det J and the basis unchanged)
    import dataclasses
    wl = st_burgers
    off = dataclasses.replace(wl, src_amp=0.0)
    mu = wl.mus[2]
    U = wl.Phi @ wl.w_eval[2]
    x = wl.X.copy()
    xs = x.reshape(-1, 2).copy()
    xs[:, 0] += 3.0
    xs = xs.reshape(-1)
    parts = []
    for xx in (x, xs):
        Rs = rs.hdm_assemble(rs.Problem(wl), mu, U, xx, jac=False)["R"]
        R0 = rs.hdm_assemble(rs.Problem(off), mu, U, xx, jac=False)["R"]
        parts.append(Rs - R0)
    assert rel(parts[1], parts[0] * np.exp(mu[1] * 3.0)) < 1e-13


def test_spacetime_boundary_data(st_burgers):
    # u = 1 everywhere, no source: with a = mu[0] = 1 every boundary value is
    # 1 and the discrete residual vanishes (free stream); with a = 4 only the
    # elements with a face on the left edge (tag 1, u = a) feel it, since the
    # bottom edge (tag 3) keeps u = 1
    import dataclasses
    wl = dataclasses.replace(st_burgers, src_amp=0.0)
    pb = rs.Problem(wl)
    U = np.ones(wl.N_u)
    R1 = rs.hdm_assemble(pb, np.array([1.0, 0.05]), U, wl.X.copy(), jac=False)["R"]
    assert np.abs(R1).max() < 1e-12
    R4 = rs.hdm_assemble(pb, np.array([4.0, 0.05]), U, wl.X.copy(), jac=False)["R"].reshape(wl.mesh.n_elem, -1)
    left = (wl.mesh.elem_nbr == -1).any(axis=1)
    assert np.abs(R4[~left]).max() < 1e-12
    assert (np.abs(R4[left]).max(axis=1) > 1e-3).all()
