"""GPU parity of the snapshot alignment (eq. (align0)) against the oracle:
device-assembled full-order Jacobian blocks, host sparse normal equations.

The device path solves the damped normal equations, the oracle the stacked
least-squares problem by dense lstsq; the two agree to about cond(M)^2 *
1e-16 (M the stacked matrix), the bound used.  Objectives are full-order
sums of squares in different orders (1e-12)."""
import sys

import numpy as np
import pytest

import synth
from conftest import rel

pytestmark = pytest.mark.gpu

LAM = 1e-2


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cases():
    return [("tiny", synth.tiny_burgers(), 3), ("euler_8x4", synth.euler_p2(nx=8, ny=4, n=20, m=10, n_s=12), 4)]


@pytest.mark.parametrize("case", [0, 1])
def test_alignment_step_matches_oracle(case):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import align as oal
    from oracle import residual as ors
    from paper_2305_15661_amd import align, ift
    ift.lib()
    name, wl, j = _cases()[case]
    prob = ift.Problem.from_workload(wl)
    Phi_j = np.linalg.qr(wl.Phi[:, :j])[0]
    al = align.Alignment(prob, Phi_j)
    opb = ors.Problem(wl)
    mu = wl.mus[1]
    w = Phi_j.T @ (wl.Phi @ wl.w_eval[1])
    x = wl.X + wl.Psi @ wl.tau_eval[1]
    _say(f"alignment {name}: objective and direction")
    Jd = al.objective(mu, w, x)
    Jo = oal.objective(opb, Phi_j, mu, w, x)
    assert abs(Jd - Jo) <= 1e-12 * Jo
    dw, dx, d = al.direction(mu, w, x, LAM)
    odw, odx, od = oal.direction(opb, Phi_j, mu, w, x, LAM)
    assert rel(d["g"], od["g"]) < 1e-12
    M = np.vstack([od["Jac"], np.hstack([np.zeros((x.size, j)), np.sqrt(LAM) * np.eye(x.size)])])
    c = np.linalg.cond(M)
    bound = max(1e-12, 1e-16 * c * c)
    _say(f"  cond(M) {c:.2e}, direction rel err {rel(np.r_[dw, dx], np.r_[odw, odx]):.2e} (bound {bound:.1e})")
    assert rel(np.r_[dw, dx], np.r_[odw, odx]) <= bound
    _say(f"alignment {name}: two steps")
    wo, xo = w, x
    for it in range(2):
        w1, x1, info = al.step(mu, w, x, LAM)
        wo1, xo1, oinfo = oal.step(opb, Phi_j, mu, wo, xo, LAM)
        _say(f"  step {it}: device {info['status']} alpha {info['alpha']} J {info['J_new']:.12e}; "
             f"oracle {oinfo['status']} alpha {oinfo['alpha']} J {oinfo['J_new']:.12e}")
        assert info["status"] == oinfo["status"] == "ok"
        assert info["n_backtrack"] == oinfo["n_backtrack"]
        assert abs(info["J_new"] - oinfo["J_new"]) <= 1e-10 * oinfo["J_old"]
        assert info["J_new"] < info["J_old"]
        # continue both from the oracle's iterate (the comparison is per step)
        w, x, wo, xo = wo1, xo1, wo1, xo1
    # the mapping basis takes the aligned displacement (eq. (greedy1))
    Psi_j = np.linalg.qr(wl.Psi[:, :3])[0]
    P1 = align.gram_schmidt_append(Psi_j, x - wl.X)
    P2 = oal.gram_schmidt_append(Psi_j, x - wl.X)
    assert np.abs(P1 - P2).max() < 1e-13 and np.abs(P1.T @ P1 - np.eye(4)).max() < 1e-13


def test_alignment_invalid_point_and_arguments():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import align as oal
    from oracle import residual as ors
    from paper_2305_15661_amd import align, ift
    wl = synth.tiny_burgers()
    prob = ift.Problem.from_workload(wl)
    Phi_j = np.linalg.qr(wl.Phi[:, :3])[0]
    al = align.Alignment(prob, Phi_j)
    w = Phi_j.T @ (wl.Phi @ wl.w_eval[0])
    x_bad = wl.X + 80.0 * (wl.Psi @ wl.tau_eval[0])      # inverted elements
    _say("alignment at an invalid point")
    assert np.isinf(al.objective(wl.mus[0], w, x_bad))
    assert np.isinf(oal.objective(ors.Problem(wl), Phi_j, wl.mus[0], w, x_bad))
    w1, x1, info = al.step(wl.mus[0], w, x_bad, LAM)
    assert info["status"] == "invalid" and np.array_equal(x1, x_bad)
    with pytest.raises(ValueError):
        al.direction(wl.mus[0], w, wl.X.copy(), 0.0)
    with pytest.raises(ValueError):
        align.Alignment(prob, Phi_j[:-1])
