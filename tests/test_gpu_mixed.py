"""Mixed precision (IFT_MIXED_BF16) on the GPU.

Assembly: element physics in FP32 and the projection on BF16 matrix cores
(each operand rounded with unit roundoff 2^-9, accumulation in FP32), Gram
and gradient accumulated in FP64.  The projected blocks therefore carry a
relative error of a few 1e-3; the objective, built from FP32 residuals,
about 1e-6.  H = M^T M carries twice the error of M (each of M's products
has two operands rounded to BF16, 2 * 2^-9, times the cancellation in the
k-sum), measured 6e-3 to 9e-3 here.  Bounds used: H and g within 2e-2
(Frobenius-relative) of the FP64 oracle, J within 1e-5.  Against the
FP32-element path with FP64 projection, the BF16 part alone is within the
same 2e-2.

Solves: a mixed batch (mixed rounds until the gradient norms reach 1e-5,
then FP64 refinement) must end within 1e-6 (relative, per instance) of the
FP64 batch and of the oracle's Levenberg-Marquardt iteration (FP64 on the
host) from the same start.  Two iterates that both meet |g| <= tol can differ by up to
|H^-1| * 2 tol, and the mapping block of H is weakly curved here, so both
solves run to tol = 1e-10 for this comparison.
"""
import numpy as np
import pytest

import synth
from conftest import rel
from oracle.eq import plain_start

pytestmark = pytest.mark.gpu

LAM = 1e-10
TOL = 1e-10


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def euler_mixed():
    import torch
    from paper_2305_15661_amd import ift
    dev = torch.device("cuda:0")
    wl = synth.euler_p2(nx=16, ny=8, n=20, m=10, n_s=64)
    prob = ift.Problem.from_workload(wl)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), device=dev)
    roms = {p: ift.ROM(prob, t(wl.Phi), t(wl.Psi), wl.eq_elem, wl.eq_rho, p) for p in ("mixed", "fp32", "fp64")}
    return dict(ift=ift, dev=dev, wl=wl, prob=prob, roms=roms)


def _jac(rom, dev, mu, w, tau):
    import torch
    J, g, H = (torch.zeros(s, dtype=torch.float64, device=dev) for s in (1, rom.D, rom.D * rom.D))
    rom.eq_assemble_jacobian(mu, torch.tensor(w, device=dev), torch.tensor(tau, device=dev), J, g, H)
    torch.cuda.synchronize()
    return J.item(), g.cpu().numpy(), H.cpu().numpy().reshape(rom.D, rom.D)


@pytest.mark.parametrize("p", [1, 2])
def test_mixed_jacobian_with_source_error_bounds(p):
    """The space-time Burgers problem with its source (the extra
    source-position rows of the mapping factor in BF16) within the same
    bounds of the FP64 oracle."""
    import torch
    from oracle import eq as oeq
    from oracle import residual as ors
    from paper_2305_15661_amd import ift
    dev = torch.device("cuda:0")
    wl = synth.spacetime_burgers(p=p) if p == 1 else synth.spacetime_burgers(nx=6, ny=6, p=2, n=6, n_s=30)
    prob = ift.Problem.from_workload(wl)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), device=dev)
    rom = ift.ROM(prob, t(wl.Phi), t(wl.Psi), wl.eq_elem, wl.eq_rho, "mixed")
    orom = oeq.ROM(ors.Problem(wl), wl.Phi, wl.Psi, wl.eq_elem, wl.eq_rho)
    for k in (0, 5, 10):
        mu, w, tau = wl.mus[k], wl.w_eval[k], wl.tau_eval[k]
        _say(f"mixed jacobian with source p{p} point {k}")
        oj = orom.jacobian(mu, w, tau)
        Jm, gm, Hm = _jac(rom, dev, mu, w, tau)
        _say(f"  rel J {abs(Jm - oj['J']) / oj['J']:.2e} g {rel(gm, oj['g']):.2e} H {rel(Hm, oj['H']):.2e}")
        assert abs(Jm - oj["J"]) <= 1e-5 * oj["J"]
        assert rel(gm, oj["g"]) < 2e-2 and rel(Hm, oj["H"]) < 2e-2


def test_mixed_jacobian_error_bounds(euler_mixed):
    from oracle import eq as oeq
    from oracle import residual as ors
    S = euler_mixed
    wl, dev = S["wl"], S["dev"]
    orom = oeq.ROM(ors.Problem(wl), wl.Phi, wl.Psi, wl.eq_elem, wl.eq_rho)
    checked = 0
    for k in range(0, 16, 3):
        mu, w, tau = wl.mus[k], wl.w_eval[k], wl.tau_eval[k]
        oj = orom.jacobian(mu, w, tau)
        if not np.isfinite(oj["J"]):
            continue
        _say(f"mixed jacobian at point {k}")
        Jm, gm, Hm = _jac(S["roms"]["mixed"], dev, mu, w, tau)
        Jf, gf, Hf = _jac(S["roms"]["fp32"], dev, mu, w, tau)
        _say(f"  rel J {abs(Jm - oj['J']) / oj['J']:.2e} g {rel(gm, oj['g']):.2e} H {rel(Hm, oj['H']):.2e}"
             f"  (fp32 elements: g {rel(gf, oj['g']):.2e} H {rel(Hf, oj['H']):.2e})")
        assert abs(Jm - oj["J"]) <= 1e-5 * oj["J"]
        assert rel(gm, oj["g"]) < 2e-2 and rel(Hm, oj["H"]) < 2e-2
        assert rel(Hm, Hf) < 2e-2 and rel(gm, gf) < 2e-2
        # the FP32-element path with FP64 projection is far closer
        assert rel(Hf, oj["H"]) < 1e-4
        checked += 1
    assert checked >= 3


def test_mixed_batched_solve_within_1e6_of_fp64():
    import torch
    from paper_2305_15661_amd import ift
    dev = torch.device("cuda:0")
    base = synth.euler_p2(nx=16, ny=8, n=30, m=10, n_s=1)
    prob = ift.Problem.from_workload(base)
    rng = np.random.default_rng(77)
    shapes = [(20, 10, 60), (10, 5, 30), (30, 10, 90), (20, 5, 45), (30, 5, 20)]
    t = lambda a: torch.tensor(np.ascontiguousarray(a), device=dev)
    from oracle import eq as oeq
    from oracle import gn as ogn
    from oracle import residual as ors
    oprob = ors.Problem(base)
    roms = {"mixed": [], "fp64": []}
    mus, starts, els, rhos = [], [], [], []
    for i, (n, m, ns) in enumerate(shapes):
        el = synth.eq_set_with_inflow(base.mesh, ns, rng)
        rho = rng.lognormal(0.0, 0.5, size=el.size)
        els.append(el)
        rhos.append(rho)
        mu = np.array([2.0 + 0.2 * i, -4.0 + 2.0 * i])
        for p in roms:
            roms[p].append(ift.ROM(prob, t(base.Phi[:, :n]), t(base.Psi[:, :m]), el, rho, p))
        w0, tau0 = plain_start(base, mu)
        mus.append(mu)
        starts.append(np.concatenate([w0[:n], tau0[:m]]))
    out = {}
    for p in roms:
        b = ift.Batch(roms[p])
        muv = torch.tensor(np.stack(mus), dtype=torch.float64, device=dev)
        z = b.pack(starts, dev)
        info = b.info_buffer(dev)
        _say(f"batched solve {p}")
        b.solve(muv, z, info, lam=LAM, max_it=150, tol=TOL)
        torch.cuda.synchronize()
        out[p] = (b.unpack(z), b.info_array(info))
    zf, inf_f = out["fp64"]
    zm, inf_m = out["mixed"]
    # an FP64 batch takes no mixed-precision steps; a mixed batch takes some,
    # and at most as many as its iterations
    assert np.all(inf_f["mixed_iterations"] == 0)
    assert np.all(inf_m["mixed_iterations"] <= inf_m["iterations"])
    assert np.sum(inf_m["mixed_iterations"]) > 0
    n_conv = 0
    for i in range(len(shapes)):
        _say(f"instance {i}: fp64 status {inf_f['status'][i]} its {inf_f['iterations'][i]}; "
             f"mixed status {inf_m['status'][i]} its {inf_m['iterations'][i]}")
        if inf_f["converged"][i]:
            assert inf_m["converged"][i] == 1
            assert inf_m["norm_S"][i] <= TOL and inf_m["norm_T"][i] <= TOL   # final check is FP64
            err = rel(zm[i], zf[i])
            n, m = shapes[i][0], shapes[i][1]
            orom = oeq.ROM(oprob, base.Phi[:, :n], base.Psi[:, :m], els[i], rhos[i])
            w, tau, oinfo = ogn.lm_solve(orom, mus[i], starts[i][:n], starts[i][n:], LAM, TOL, 150)
            zo = np.r_[w, tau]
            err_o, err_fo = rel(zm[i], zo), rel(zf[i], zo)
            _say(f"  relative state error vs FP64 batch {err:.2e}, vs oracle {err_o:.2e} (FP64 batch vs oracle "
                 f"{err_fo:.2e}; oracle {oinfo['status']} in {oinfo['iterations']} steps)")
            assert oinfo["status"] == "converged"
            assert err <= 1e-6 and err_o <= 1e-6 and err_fo <= 1e-6
            n_conv += 1
    assert n_conv >= 3
