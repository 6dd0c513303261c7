"""EQ-weight training (eq. (eqp-lp)-(eqp-con)) on the host, with the
elemental reduced residuals of the oracle: the oracle's elemental terms are
pinned to its assembled gradient and to single-element EQ sets; the program
is feasible at rho = 1 (the paper's remark on the feasible set), its
solution meets every constraint, is sparse, and its weighted reduced
residuals match the full ones at the training solutions."""
import numpy as np

from oracle import eq
from oracle import residual as rs
from paper_2305_15661_amd import eqp


def _all_elements_rom(wl, rho=None):
    Ne = wl.mesh.n_elem
    el = np.arange(Ne, dtype=np.int32)
    return eq.ROM(rs.Problem(wl), wl.Phi, wl.Psi, el, np.ones(Ne) if rho is None else rho)


def test_element_contributions_sum_to_gradient_and_match_single_elements(tiny):
    wl = tiny
    rom = eq.ROM(rs.Problem(wl), wl.Phi, wl.Psi, wl.eq_elem, wl.eq_rho)
    mu, w, tau = wl.mus[2], wl.w_eval[2], wl.tau_eval[2]
    C = rom.element_contributions(mu, w, tau)
    g = rom.jacobian(mu, w, tau)["g"]
    assert np.linalg.norm(wl.eq_rho @ C - g) <= 1e-13 * np.linalg.norm(g)
    for k in (0, 7, 19):
        one = eq.ROM(rs.Problem(wl), wl.Phi, wl.Psi, wl.eq_elem[k:k + 1], np.ones(1))
        gk = one.jacobian(mu, w, tau)["g"]
        assert np.linalg.norm(C[k] - gk) <= 1e-13 * max(np.linalg.norm(gk), 1e-300)


def test_element_volumes_sum_to_domain(tiny):
    wl = tiny
    vol = eqp.element_volumes(wl.mesh.X, wl.mesh.elem_gnodes)
    assert vol.size == wl.mesh.n_elem and np.all(vol > 0)
    assert abs(vol.sum() - 1.0) < 1e-14          # the unit square


def test_training_program_feasible_sparse_and_accurate(tiny):
    wl = tiny
    rom = _all_elements_rom(wl)
    Ne = wl.mesh.n_elem
    train = [(wl.mus[k], wl.w_eval[k], wl.tau_eval[k]) for k in (1, 5, 9)]
    contribs = [rom.element_contributions(*t) for t in train]
    vol = eqp.element_volumes(wl.mesh.X, wl.mesh.elem_gnodes)
    scale = max(np.abs(C.sum(axis=0)).max() for C in contribs)
    delta = 1e-2 * scale
    c, A, b = eqp.program(contribs, vol, delta)
    assert np.all(A @ np.ones(Ne) <= b + 1e-12)                  # rho = 1 is feasible
    rho, info = eqp.train_weights(contribs, vol, delta)
    assert info["status"] == 0
    assert np.all(rho >= 0) and info["max_violation"] <= 1e-9
    assert info["objective"] <= Ne + 1e-9 and info["nnz"] < Ne
    # the weighted reduced residuals of an EQ set of the nonzero weights
    nz = np.nonzero(rho)[0].astype(np.int32)
    erom = eq.ROM(rs.Problem(wl), wl.Phi, wl.Psi, nz, rho[nz])
    for (mu, w, tau), C in zip(train, contribs):
        full = C.sum(axis=0)
        g = erom.jacobian(mu, w, tau)["g"]
        assert np.max(np.abs(g - full)) <= delta / len(train) * (1 + 1e-8) + 1e-12
    assert abs(vol @ rho - vol.sum()) <= delta * vol.sum() * (1 + 1e-8)


def test_program_targets_the_unweighted_sums_for_any_guess(tiny):
    """With a guess rho_check != 1 the training solutions move, but the
    accuracy constraints still compare with the unweighted all-element sums
    (the hatted S, T of eq. (eqp-con)): rho = 1 stays feasible, while the
    guess itself is not (its weighted sums miss the unweighted ones by far
    more than delta)."""
    wl = tiny
    Ne = wl.mesh.n_elem
    rng = np.random.default_rng(17)
    rho_check = np.where(rng.random(Ne) < 0.3, rng.uniform(0.5, 3.0, Ne), 0.0)
    rom = _all_elements_rom(wl)
    train = [(wl.mus[k], wl.w_eval[k], wl.tau_eval[k]) for k in (2, 6)]
    contribs = [rom.element_contributions(*t) for t in train]
    vol = eqp.element_volumes(wl.mesh.X, wl.mesh.elem_gnodes)
    scale = max(np.abs(C.sum(axis=0)).max() for C in contribs)
    delta = 1e-3 * scale
    c, A, b = eqp.program(contribs, vol, delta, delta_vol=10.0)
    assert np.all(A @ np.ones(Ne) <= b + 1e-12)
    assert np.max(A @ rho_check - b) > 1.0
