"""GPU parity: every output of the HIP path against the CPU oracle on the
same seeded inputs, through the C ABI.

Tolerances (FP64): normwise relative error <= 1e-12 for residuals,
Jacobians, gradients and Gauss-Newton matrices (both sides compute the same
sums of O(10^2) terms in a different order; the observed error is ~1e-15);
gathers are bit-exact; a Gauss-Newton step is compared given the same z_n
with a bound of 1e-13 * cond(H) (the two sides factor H independently)."""
import sys

import numpy as np
import pytest

import synth
from conftest import gram_entry_err, rel, rel_blocks

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_15661_amd import ift
    ift.lib()            # fails loudly if the HIP library is missing
    return torch.device("cuda:0")


def _t(a, dev):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def _z(n, dev, dtype=None):
    import torch
    return torch.zeros(n, dtype=dtype or torch.float64, device=dev)


class Case:
    def __init__(self, wl, dev, eq_elem=None, eq_rho=None, precision="fp64"):
        from oracle import eq as oeq
        from oracle import residual as ors
        from paper_2305_15661_amd import ift
        self.wl = wl
        self.dev = dev
        self.eq_elem = wl.eq_elem if eq_elem is None else np.asarray(eq_elem, dtype=np.int32)
        self.eq_rho = wl.eq_rho if eq_rho is None else np.asarray(eq_rho)
        self.prob = ift.Problem.from_workload(wl)
        self.rom = ift.ROM(self.prob, _t(wl.Phi, dev), _t(wl.Psi, dev), self.eq_elem, self.eq_rho, precision)
        self.oprob = ors.Problem(wl)
        self.orom = oeq.ROM(self.oprob, wl.Phi, wl.Psi, self.eq_elem, self.eq_rho)


@pytest.fixture(scope="module")
def tiny_case(dev):
    return Case(synth.tiny_burgers(), dev)


@pytest.fixture(scope="module")
def st_case(dev):
    # the space-time Burgers problem with its source, 8x8 P1 cells
    return Case(synth.spacetime_burgers(), dev)


@pytest.fixture(scope="module")
def st_p2_case(dev):
    # the same on 6x6 P2 cells (curved elements), 30 EQ elements
    return Case(synth.spacetime_burgers(nx=6, ny=6, p=2, n=6, n_s=30), dev)


@pytest.fixture(scope="module")
def euler_p1_case(dev):
    # P1 Euler, 16x8 cells, 64 EQ elements (the other four-component discretisation)
    return Case(synth.euler_p2(nx=16, ny=8, n=20, m=10, n_s=64, p=1), dev)


@pytest.fixture(scope="module")
def euler_case(dev):
    # 16x8 cells (256 P2 elements), 64 EQ elements: several tiles and a ragged tail
    return Case(synth.euler_p2(nx=16, ny=8, n=20, m=10, n_s=64), dev)


@pytest.fixture(scope="module")
def euler_odd_case(dev):
    # an odd element count and an odd EQ set: the 16x8 P2 mesh without its
    # last element (the face it shared becomes a top-boundary face), so the
    # kernels that take two elements per block run their one-element tail
    import dataclasses
    wl = synth.euler_p2(nx=16, ny=8, n=20, m=10, n_s=64)
    m = wl.mesh
    Ne = m.n_elem
    nbr = m.elem_nbr[:-1].copy()
    nbr[nbr == Ne - 1] = -4
    mesh = dataclasses.replace(m, elem_gnodes=m.elem_gnodes[:-1].copy(), elem_nbr=nbr)
    nue = wl.Phi.shape[0] // Ne
    keep = np.nonzero(wl.eq_elem < Ne - 1)[0]
    if keep.size % 2 == 0:
        keep = keep[1:]
    wl = dataclasses.replace(wl, name=wl.name + "-odd", mesh=mesh, Phi=wl.Phi[:-nue].copy(),
                             eq_elem=wl.eq_elem[keep].copy(), eq_rho=wl.eq_rho[keep].copy())
    assert mesh.n_elem % 2 == 1 and wl.eq_elem.size % 2 == 1
    return Case(wl, dev)


def _hdm_gpu(case, mu, U, x, jac=True):
    import torch
    p, d = case.prob, case.dev
    Ne = p.n_elem
    out = {"R": _z(p.N_u, d), "N": _z(Ne, d), "n_bad": _z(1, d, torch.int32)}
    if jac:
        out.update(dRdU=_z(Ne * p.nue * p.nue, d), dRdUn=_z(Ne * p.nue * p.nun, d),
                   dRdx=_z(Ne * p.nue * p.nxe, d), dNdx=_z(Ne * p.nxe, d))
    p.hdm_assemble(mu, _t(U, d), _t(x, d), **out)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("which", ["tiny_case", "euler_case", "st_case", "st_p2_case", "euler_p1_case",
                                   "euler_odd_case"])
def test_hdm_assemble_parity(which, request):
    from oracle import residual as ors
    case = request.getfixturevalue(which)
    wl = case.wl
    for k in (0, 7):
        _say(f"hdm_assemble parity {wl.name} eval point {k}")
        mu = wl.mus[k]
        U = wl.Phi @ wl.w_eval[k]
        x = wl.X + wl.Psi @ wl.tau_eval[k]
        g = _hdm_gpu(case, mu, U, x)
        o = ors.hdm_assemble(case.oprob, mu, U, x, jac=True)
        assert rel(g["R"], o["R"]) < 1e-12
        assert rel(g["N"], o["N"]) < 1e-12
        for key in ("dRdU", "dRdUn", "dRdx", "dNdx"):
            assert rel(g[key], o[key].ravel()) < 1e-12, key
        # element by element: R_e and every Jacobian block on its own scale
        Ne = wl.mesh.n_elem
        for key, ref in (("R", o["R"]), ("dRdU", o["dRdU"]), ("dRdUn", o["dRdUn"]), ("dRdx", o["dRdx"]),
                         ("dNdx", o["dNdx"])):
            assert rel_blocks(g[key], ref, Ne) < 1e-11, key
        # N_e is a difference of two integrals of size ~4 kappa |Omega_e|:
        # its rounding is bounded on that scale, element by element
        X = wl.mesh.X.reshape(-1, 2)
        area_e = np.ptp(X[:, 0]) * np.ptp(X[:, 1]) / Ne
        assert np.abs(g["N"] - o["N"]).max() <= 1e-12 * 4.0 * wl.kappa * area_e
        assert int(g["n_bad"][0]) == o["n_bad"] == 0


def test_hdm_residual_only_matches_jacobian_path(euler_case):
    wl = euler_case.wl
    U = wl.Phi @ wl.w_eval[3]
    x = wl.X + wl.Psi @ wl.tau_eval[3]
    a = _hdm_gpu(euler_case, wl.mus[3], U, x, jac=False)
    b = _hdm_gpu(euler_case, wl.mus[3], U, x, jac=True)
    # the Jacobian path evaluates the point values in tangent arithmetic,
    # which the compiler may contract differently: equal to rounding.  N_e is
    # a difference of two integrals of size ~4|Omega_e| kappa, so its
    # rounding error scales with that size, not with N_e.
    assert rel(a["R"], b["R"]) < 1e-14
    eta_scale = wl.kappa * 4.0 * (2.0 / wl.mesh.n_elem)
    assert np.abs(a["N"] - b["N"]).max() < 1e-14 * eta_scale


@pytest.mark.parametrize("which", ["tiny_case", "euler_case", "st_case", "st_p2_case"])
def test_gathers_bit_exact(which, request):
    case = request.getfixturevalue(which)
    _say(f"gathers {case.wl.name}")
    p, r, d = case.prob, case.rom, case.dev
    bufs = [_z(r.n_s * p.nue * r.n, d), _z(r.n_s * p.nun * r.n, d), _z(r.n_s * p.nxe * r.m, d), _z(r.n_s * p.nxe, d)]
    r.get_gathers(*bufs)
    o = case.orom
    for b, ref in zip(bufs, (o.Phi_s, o.Phin_s, o.Psi_s, o.X_s)):
        assert np.array_equal(b.cpu().numpy(), ref.ravel())


def _eq_gpu(case, mu, w, tau):
    import torch
    r, d = case.rom, case.dev
    J, g, H, Jt = _z(1, d), _z(r.D, d), _z(r.D * r.D, d), _z(r.nrows * r.D, d)
    nb = _z(1, d, torch.int32)
    r.eq_assemble_jacobian(mu, _t(w, d), _t(tau, d), J, g, H, Jt, nb)
    Jr, Ft, ptr, nb2 = _z(1, d), _z(r.nrows, d), _z(r.n, d), _z(1, d, torch.int32)
    r.eq_assemble_residual(mu, _t(w, d), _t(tau, d), Jr, Ft, ptr, nb2)
    torch.cuda.synchronize()
    f = lambda t: t.cpu().numpy()
    return dict(J=f(J)[0], g=f(g), H=f(H).reshape(r.D, r.D), Jt=f(Jt).reshape(r.nrows, r.D), Jr=f(Jr)[0],
                Ft=f(Ft), PhiT_r=f(ptr), n_bad=int(f(nb)[0]))


@pytest.mark.parametrize("which", ["tiny_case", "euler_case", "st_case", "st_p2_case", "euler_p1_case",
                                   "euler_odd_case"])
def test_eq_assembly_parity(which, request):
    case = request.getfixturevalue(which)
    wl = case.wl
    for k in range(0, 16, 5):
        _say(f"eq assembly parity {wl.name} eval point {k}")
        mu, w, tau = wl.mus[k], wl.w_eval[k], wl.tau_eval[k]
        g = _eq_gpu(case, mu, w, tau)
        oj = case.orom.jacobian(mu, w, tau)
        orr = case.orom.residual(mu, w, tau)
        assert abs(g["J"] - oj["J"]) <= 1e-12 * oj["J"]
        assert abs(g["Jr"] - oj["J"]) <= 1e-12 * oj["J"]
        assert rel(g["g"], oj["g"]) < 1e-12
        assert rel(g["H"], oj["H"]) < 1e-12
        eH, eg = gram_entry_err(g["H"].reshape(oj["H"].shape), g["g"], oj["H"], oj["g"], oj["J"])
        assert eH < 1e-12 and eg < 1e-12, (eH, eg)
        assert rel(g["Jt"], oj["Jt"]) < 1e-12
        nr = case.rom.n_s * case.prob.nue
        assert rel_blocks(g["Jt"][:nr], oj["Jt"][:nr], case.rom.n_s) < 1e-11
        assert rel(g["Ft"], orr["Ft"]) < 1e-12
        assert rel(g["PhiT_r"], orr["PhiT_r"]) < 1e-12
        assert g["n_bad"] == 0


def test_eq_assembly_is_deterministic(euler_case):
    wl = euler_case.wl
    a = _eq_gpu(euler_case, wl.mus[1], wl.w_eval[1], wl.tau_eval[1])
    b = _eq_gpu(euler_case, wl.mus[1], wl.w_eval[1], wl.tau_eval[1])
    for k in ("g", "H", "Jt", "Ft"):
        assert np.array_equal(a[k], b[k])
    assert a["J"] == b["J"]


def test_invalid_point_reported(tiny_case):
    wl = tiny_case.wl
    _say("invalid evaluation point")
    g = _eq_gpu(tiny_case, wl.mus[0], wl.w_eval[0], 80.0 * wl.tau_eval[0])
    o = tiny_case.orom.residual(wl.mus[0], wl.w_eval[0], 80.0 * wl.tau_eval[0])
    assert np.isinf(g["J"]) and np.isinf(g["Jr"]) and o["invalid"]
    assert g["n_bad"] == o["n_bad"] > 0


def test_single_element_and_boundary_only_eq_sets(dev):
    wl = synth.euler_p2(nx=8, ny=4, n=20, m=10, n_s=12)
    for el in ([5], np.nonzero((wl.mesh.elem_nbr < 0).any(axis=1))[0]):
        _say(f"eq set of size {len(el)}")
        case = Case(wl, dev, eq_elem=el, eq_rho=np.linspace(0.5, 1.5, len(el)))
        mu, w, tau = wl.mus[2], wl.w_eval[2], wl.tau_eval[2]
        g = _eq_gpu(case, mu, w, tau)
        oj = case.orom.jacobian(mu, w, tau)
        assert rel(g["g"], oj["g"]) < 1e-12 and rel(g["H"], oj["H"]) < 1e-12


@pytest.mark.parametrize("which", ["tiny_case", "euler_case", "st_case", "st_p2_case", "euler_p1_case",
                                   "euler_odd_case"])
def test_batched_points_match_single_calls_and_oracle(which, request):
    """All 16 seeded evaluation points in one batched launch (device mu)."""
    import torch
    case = request.getfixturevalue(which)
    wl, r, d = case.wl, case.rom, case.dev
    P = wl.mus.shape[0]
    _say(f"batched eq assembly {wl.name} x{P}")
    r.reserve(P)
    mu2 = np.zeros((P, 2))
    mu2[:, :wl.mus.shape[1]] = wl.mus
    MU, W, T = _t(mu2, d), _t(wl.w_eval, d), _t(wl.tau_eval, d)
    J, G, H = _z(P, d), _z(P * r.D, d), _z(P * r.D * r.D, d)
    nb = _z(P, d, torch.int32)
    r.eq_assemble_jacobian_batch(MU, W, T, J, G, H, nb)
    Jr = _z(P, d)
    r.eq_assemble_residual_batch(MU, W, T, Jr)
    torch.cuda.synchronize()
    J, G, H, Jr = J.cpu().numpy(), G.cpu().numpy().reshape(P, r.D), H.cpu().numpy().reshape(P, r.D, r.D), Jr.cpu().numpy()
    for k in (0, 5, P - 1):
        single = _eq_gpu(case, wl.mus[k], wl.w_eval[k], wl.tau_eval[k])
        oj = case.orom.jacobian(wl.mus[k], wl.w_eval[k], wl.tau_eval[k])
        assert rel(G[k], single["g"]) < 1e-14 and rel(H[k], single["H"]) < 1e-14
        assert rel(G[k], oj["g"]) < 1e-12 and rel(H[k], oj["H"]) < 1e-12
        assert abs(J[k] - oj["J"]) <= 1e-12 * oj["J"] and abs(Jr[k] - oj["J"]) <= 1e-12 * oj["J"]
    nb_o = [case.orom.residual(wl.mus[k], wl.w_eval[k], wl.tau_eval[k])["n_bad"] for k in range(P)]
    assert list(nb.cpu().numpy()) == nb_o
    assert all(np.isinf(J[k]) == (nb_o[k] > 0) for k in range(P))


@pytest.mark.parametrize("P", [2, 7])
def test_batched_points_pairs_and_lone_point(P, euler_case):
    """Multi-point FP64 calls of the P2 Euler ROM take two points of an element
    per wave; an odd point count leaves a lone last point.  Every point
    against its single call and the oracle."""
    import torch
    case = euler_case
    wl, r, d = case.wl, case.rom, case.dev
    idx = [3, 0, 11, 5, 15, 8, 1][:P]
    _say(f"batched eq assembly {wl.name} x{P} (stacked points)")
    r.reserve(P)
    mu2 = np.zeros((P, 2))
    mu2[:, :wl.mus.shape[1]] = wl.mus[idx]
    MU, W, T = _t(mu2, d), _t(wl.w_eval[idx], d), _t(wl.tau_eval[idx], d)
    J, G, H = _z(P, d), _z(P * r.D, d), _z(P * r.D * r.D, d)
    nb = _z(P, d, torch.int32)
    r.eq_assemble_jacobian_batch(MU, W, T, J, G, H, nb)
    torch.cuda.synchronize()
    J, G, H = J.cpu().numpy(), G.cpu().numpy().reshape(P, r.D), H.cpu().numpy().reshape(P, r.D, r.D)
    for j, k in enumerate(idx):
        single = _eq_gpu(case, wl.mus[k], wl.w_eval[k], wl.tau_eval[k])
        oj = case.orom.jacobian(wl.mus[k], wl.w_eval[k], wl.tau_eval[k])
        assert rel(G[j], single["g"]) < 1e-14 and rel(H[j], single["H"]) < 1e-14
        assert rel(G[j], oj["g"]) < 1e-12 and rel(H[j], oj["H"]) < 1e-12
        if np.isinf(oj["J"]):
            assert np.isinf(J[j])
        else:
            assert abs(J[j] - oj["J"]) <= 1e-12 * oj["J"]
        assert nb.cpu().numpy()[j] == single["n_bad"]


@pytest.mark.parametrize("n,m,n_s", [(12, 12, 64), (8, 4, 64), (21, 10, 64), (20, 10, 3)])
def test_batched_points_column_tiles(n, m, n_s, dev):
    """Multi-point FP64 calls across the stacked-point kernel's column-tile
    cases: two tiles with n <= 16 (every tile reached), one tile, and
    n + m = 31, which the one-point kernel takes; and three sampled elements,
    which leave most of its blocks without an element.  Five points (two
    pairs and a lone point), each against its single call and the oracle."""
    import torch
    case = Case(synth.euler_p2(nx=16, ny=8, n=n, m=m, n_s=n_s), dev)
    wl, r, d = case.wl, case.rom, case.dev
    idx = [3, 0, 11, 5, 8]
    P = len(idx)
    _say(f"batched eq assembly n={n} m={m} n_s={n_s} x{P}")
    r.reserve(P)
    mu2 = np.zeros((P, 2))
    mu2[:, :wl.mus.shape[1]] = wl.mus[idx]
    MU, W, T = _t(mu2, d), _t(wl.w_eval[idx], d), _t(wl.tau_eval[idx], d)
    J, G, H = _z(P, d), _z(P * r.D, d), _z(P * r.D * r.D, d)
    nb = _z(P, d, torch.int32)
    r.eq_assemble_jacobian_batch(MU, W, T, J, G, H, nb)
    torch.cuda.synchronize()
    J, G, H = J.cpu().numpy(), G.cpu().numpy().reshape(P, r.D), H.cpu().numpy().reshape(P, r.D, r.D)
    for j, k in enumerate(idx):
        single = _eq_gpu(case, wl.mus[k], wl.w_eval[k], wl.tau_eval[k])
        oj = case.orom.jacobian(wl.mus[k], wl.w_eval[k], wl.tau_eval[k])
        assert nb.cpu().numpy()[j] == single["n_bad"]
        if np.isinf(oj["J"]):   # an invalid lifted state: J~ = +inf, counted
            assert np.isinf(J[j]) and single["n_bad"] > 0
            continue
        assert single["n_bad"] == 0
        assert rel(G[j], single["g"]) < 1e-14 and rel(H[j], single["H"]) < 1e-14
        assert rel(G[j], oj["g"]) < 1e-12 and rel(H[j], oj["H"]) < 1e-12
        assert abs(J[j] - oj["J"]) <= 1e-12 * oj["J"]


@pytest.mark.parametrize("which", ["tiny_case", "st_case"])
def test_gauss_newton_steps_parity(which, request):
    """Twenty steps from the plain start; each GPU step is compared with the
    oracle's step from the same z_n (normal equations, Armijo backtracking)."""
    import torch
    from oracle import eq as oeq
    from oracle import gn as ogn
    case = request.getfixturevalue(which)
    wl, d = case.wl, case.dev
    mu = wl.mus[0]
    w0, t0 = oeq.plain_start(wl, mu)
    z = np.r_[w0, t0]
    n = wl.n
    for it in range(20):
        _say(f"gauss-newton step {it}")
        w, tau = _t(z[:n], d), _t(z[n:], d)
        st, info = case.rom.gauss_newton_step(mu, w, tau)
        z_gpu = np.r_[w.cpu().numpy(), tau.cpu().numpy()]
        wo, to, oinfo = ogn.gn_step(case.orom, mu, z[:n], z[n:])
        assert st == 0 and oinfo["status"] in ("ok", "converged")
        assert info["n_backtrack"] == oinfo["n_backtrack"]
        H = case.orom.jacobian(mu, z[:n], z[n:])["H"]
        bound = max(1e-12, 1e-13 * np.linalg.cond(H))
        step_o = np.r_[wo, to] - z
        assert np.linalg.norm(z_gpu - np.r_[wo, to]) <= bound * max(np.linalg.norm(step_o), 1e-300) + 1e-14 * np.linalg.norm(z)
        assert abs(info["J_new"] - oinfo["J_new"]) <= 1e-10 * oinfo["J_old"]
        z = np.r_[wo, to]


@pytest.mark.parametrize("which,lam", [("tiny_case", 0.0), ("euler_case", 1e-3), ("st_p2_case", 1e-3)])
def test_gauss_newton_qr_step_parity(which, lam, request):
    """The least-squares form of the step (Householder QR of the stacked rows
    [J~_z | -F~] and, for lambda > 0, the sqrt(lambda) rows of the mapping
    block; the 20475-row benchmark case needs three reduction levels, these
    cases one or two) against the oracle's lstsq step from the same z_n, and
    against the normal-equation step of the GPU.  The two solvers agree to
    about cond(H) * 1e-16 in the direction; the bound is 1e-13 cond(H)."""
    import torch
    from oracle import gn as ogn
    case = request.getfixturevalue(which)
    wl, d = case.wl, case.dev
    n = wl.n
    checked = 0
    for k in range(4):
        mu, w, tau = wl.mus[k], wl.w_eval[k], wl.tau_eval[k]
        oj = case.orom.jacobian(mu, w, tau)
        if not np.isfinite(oj["J"]):
            continue
        _say(f"qr step at point {k}")
        wq, tq = _t(w, d), _t(tau, d)
        st, info = case.rom.gauss_newton_step(mu, wq, tq, lam=lam, qr=True)
        wc, tc = _t(w, d), _t(tau, d)
        st_c, info_c = case.rom.gauss_newton_step(mu, wc, tc, lam=lam)
        wo, to, oinfo = ogn.gn_step(case.orom, mu, w, tau, lam=lam, solver="qr")
        assert oinfo["status"] in ("ok", "linesearch")
        assert st == (0 if oinfo["status"] == "ok" else -7) and st_c == st
        assert info["n_backtrack"] == oinfo["n_backtrack"] == info_c["n_backtrack"]
        Hl = oj["H"].copy()
        Hl[n:, n:] += lam * np.eye(Hl.shape[0] - n)
        bound = max(1e-12, 1e-13 * np.linalg.cond(Hl))
        z0 = np.r_[w, tau]
        zo = np.r_[wo, to]
        zq = np.r_[wq.cpu().numpy(), tq.cpu().numpy()]
        zc = np.r_[wc.cpu().numpy(), tc.cpu().numpy()]
        step = max(np.linalg.norm(zo - z0), 1e-300)
        assert np.linalg.norm(zq - zo) <= bound * step + 1e-14 * np.linalg.norm(z0)
        assert np.linalg.norm(zq - zc) <= bound * step + 1e-14 * np.linalg.norm(z0)
        assert abs(info["norm_S"] - oinfo["norm_S"]) <= 1e-10 * max(oinfo["norm_S"], 1e-300)
        checked += 1
    assert checked >= 2


@pytest.mark.parametrize("qr", [False, True])
def test_gauss_newton_w_only_step_parity(tiny_case, qr):
    """Steps of the paper's initialisation (w with tau held, converged on
    |S~| alone) from the plain start, each compared with the oracle's w-only
    step from the same w_n (bound as for the full step, with cond(H_ww))."""
    from oracle import eq as oeq
    from oracle import gn as ogn
    case = tiny_case
    wl, d = case.wl, case.dev
    mu = wl.mus[0]
    w, tau0 = oeq.plain_start(wl, mu)
    n = wl.n
    for it in range(12):
        _say(f"w-only step {it} (qr={qr})")
        wg, tg = _t(w, d), _t(tau0, d)
        st, info = case.rom.gauss_newton_step(mu, wg, tg, qr=qr, w_only=True)
        wo, to, oinfo = ogn.gn_step(case.orom, mu, w, tau0, solver="qr" if qr else "normal", w_only=True)
        assert np.array_equal(tg.cpu().numpy(), tau0) and np.array_equal(to, tau0)
        if oinfo["status"] == "converged":
            assert st == 0 and info["converged"] == 1
            break
        assert st == 0 and oinfo["status"] == "ok"
        assert info["n_backtrack"] == oinfo["n_backtrack"]
        H = case.orom.jacobian(mu, w, tau0)["H"][:n, :n]
        bound = max(1e-12, 1e-13 * np.linalg.cond(H))
        step = max(np.linalg.norm(wo - w), 1e-300)
        assert np.linalg.norm(wg.cpu().numpy() - wo) <= bound * step + 1e-14 * np.linalg.norm(w)
        w = wo
    else:
        raise AssertionError("the w-only iteration did not converge in 12 steps")


@pytest.mark.parametrize("which", ["tiny_case", "euler_case", "st_case", "st_p2_case"])
def test_hdm_residual_norms_match_oracle(which, request):
    """The greedy indicator, eq. (greedy0): |R(Phi w; X + Psi tau, mu)|_2 over
    all elements for several reduced points in one call, against the norm of
    the oracle's full-order residual; an invalid point reports +inf and its
    invalid elements; the argmax is the same candidate."""
    import torch
    from oracle import residual as ors
    from paper_2305_15661_amd import ift
    case = request.getfixturevalue(which)
    wl, d = case.wl, case.dev
    ks = [0, 3, 6, 9]
    mu2 = lambda v: np.r_[np.atleast_1d(v), 0.0][:2]          # [n_pts][2] layout (Burgers uses mu[0])
    mus = np.stack([mu2(wl.mus[k]) for k in ks] + [mu2(wl.mus[0])])
    ws = np.stack([wl.w_eval[k] for k in ks] + [wl.w_eval[0]])
    taus = np.stack([wl.tau_eval[k] for k in ks] + [80.0 * wl.tau_eval[0]])
    P = len(mus)
    norms, nb = _z(P, d), _z(P, d, torch.int32)
    _say(f"residual norms {wl.name}")
    case.prob.hdm_residual_norms(_t(mus, d), _t(wl.Phi, d), _t(ws, d), _t(wl.Psi, d), _t(taus, d), norms, nb)
    torch.cuda.synchronize()
    g, gb = norms.cpu().numpy(), nb.cpu().numpy()
    ref = []
    for p in range(P):
        mu_o = wl.mus[ks[p]] if p < len(ks) else wl.mus[0]
        o = ors.hdm_assemble(case.oprob, mu_o, wl.Phi @ ws[p], wl.X + wl.Psi @ taus[p], jac=False)
        if o["n_bad"]:
            assert np.isinf(g[p]) and gb[p] == o["n_bad"] > 0
            ref.append(np.inf)
        else:
            r = np.linalg.norm(o["R"])
            assert abs(g[p] - r) <= 1e-12 * r and gb[p] == 0
            ref.append(r)
    assert np.isinf(ref[-1])
    assert ift.greedy_select(g[:-1]) == int(np.argmax(ref[:-1]))


@pytest.mark.parametrize("which", ["tiny_case", "euler_case", "st_case", "st_p2_case"])
def test_element_contributions_match_oracle(which, request):
    """The data of the EQ-weight training program: unweighted elemental
    reduced residuals against the oracle's (1e-12), and sum_k rho_k C[k]
    equal to the device gradient."""
    import torch
    case = request.getfixturevalue(which)
    wl, d, r = case.wl, case.dev, case.rom
    for k in (2, 11):
        mu, w, tau = wl.mus[k], wl.w_eval[k], wl.tau_eval[k]
        _say(f"element contributions {wl.name} point {k}")
        C = _z(r.n_s * r.D, d)
        r.element_contributions(mu, _t(w, d), _t(tau, d), C)
        g = _eq_gpu(case, mu, w, tau)["g"]
        torch.cuda.synchronize()
        Cg = C.cpu().numpy().reshape(r.n_s, r.D)
        Co = case.orom.element_contributions(mu, w, tau)
        assert rel(Cg, Co) < 1e-12
        assert rel(case.eq_rho @ Cg, g) < 1e-12


def test_full_size_euler_samples(dev):
    """16384 P2 elements, 819 EQ elements, n = 20, m = 10 (the benchmark
    shape): full EQ assembly against the oracle, and the full-order residual
    on a sample of elements (every 97th plus all boundary-adjacent ones of
    the first rows) computed element by element by the oracle."""
    import torch
    wl = synth.euler_p2()
    case = Case(wl, dev)
    k = 4
    mu, w, tau = wl.mus[k], wl.w_eval[k], wl.tau_eval[k]
    _say("full size: eq assembly")
    g = _eq_gpu(case, mu, w, tau)
    oj = case.orom.jacobian(mu, w, tau)
    assert rel(g["g"], oj["g"]) < 1e-12 and rel(g["H"], oj["H"]) < 1e-12
    assert abs(g["J"] - oj["J"]) <= 1e-12 * oj["J"]
    _say("full size: hdm_assemble residual + jacobians on sampled elements")
    U = wl.Phi @ w
    x = wl.X + wl.Psi @ tau
    gg = _hdm_gpu(case, mu, U, x, jac=True)
    Ne = wl.mesh.n_elem
    el = np.unique(np.r_[np.arange(0, Ne, 97), np.arange(0, 256), np.arange(Ne - 256, Ne)])
    o = case.oprob.evaluate(el, *case.oprob.gather_state(el, U, x), mu, jac=True)
    p = case.prob
    assert rel(gg["R"].reshape(Ne, -1)[el], o["R"]) < 1e-12
    assert rel(gg["N"][el], o["N"]) < 1e-12
    assert rel(gg["dRdU"].reshape(Ne, p.nue, p.nue)[el], o["dRdU"]) < 1e-12
    assert rel(gg["dRdUn"].reshape(Ne, p.nue, p.nun)[el], o["dRdUn"]) < 1e-12
    assert rel(gg["dRdx"].reshape(Ne, p.nue, p.nxe)[el], o["dRdx"]) < 1e-12
    del gg
    torch.cuda.empty_cache()


def test_plain_start_burgers_matches_oracle(tiny_case):
    import torch
    from oracle.eq import plain_start
    case = tiny_case
    wl, r, d = case.wl, case.rom, case.dev
    for mu in (wl.mus[0], np.array([0.9, 0.0])):
        _say(f"plain start burgers mu={mu}")
        w, tau = _z(r.n, d), _z(r.m, d)
        r.plain_start(mu, w, tau)
        torch.cuda.synchronize()
        w0, t0 = plain_start(wl, mu)
        assert rel(w.cpu().numpy(), w0) < 1e-13 and np.all(tau.cpu().numpy() == t0)
