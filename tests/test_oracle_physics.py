"""Pins of the oracle's fluxes: consistency, Roe's property, conservation
symmetry, homogeneity, rotational invariance and exact derivatives."""
import numpy as np
import pytest

from oracle import physics as ph
from oracle.dual import Dual

G = 1.4


def _states(rng, k):
    rho = rng.uniform(0.5, 2.0, k)
    vx, vy = rng.uniform(-2, 2, k), rng.uniform(-2, 2, k)
    p = rng.uniform(0.5, 2.0, k)
    return np.stack([rho, rho * vx, rho * vy, p / (G - 1) + 0.5 * rho * (vx ** 2 + vy ** 2)], axis=1)


def test_euler_flux_closed_form():
    u = np.array([1.2, 0.6, -0.3, 3.0])
    rho, vx, vy, E = 1.2, 0.5, -0.25, 3.0
    p = 0.4 * (E - 0.5 * rho * (vx ** 2 + vy ** 2))
    f = ph.euler_flux(u, G).v
    ref = np.array([[rho * vx, rho * vy], [rho * vx ** 2 + p, rho * vx * vy],
                    [rho * vx * vy, rho * vy ** 2 + p], [(E + p) * vx, (E + p) * vy]])
    assert np.abs(f - ref).max() < 1e-15


def test_roe_property_and_consistency():
    rng = np.random.default_rng(1)
    uL, uR = _states(rng, 50), _states(rng, 50)
    th = rng.uniform(0, 2 * np.pi, 50)
    n = np.stack([np.cos(th), np.sin(th)], axis=1)
    lams, als, rs, _ = ph.roe_waves(uL, uR, n, G)
    s = sum(l.v[:, None] * a.v[:, None] * r.v for l, a, r in zip(lams, als, rs))
    fn = lambda u: np.einsum("kcd,kd->kc", ph.euler_flux(u, G).v, n)
    assert np.abs(s - (fn(uR) - fn(uL))).max() < 1e-12
    # eigenvectors: A r_k = lam_k r_k for the Roe matrix at uL = uR
    H = ph.euler_roe(uL, uL, 3.0 * n, G).v
    assert np.abs(H - 3.0 * fn(uL)).max() < 1e-12


def test_roe_conservation_homogeneity_rotation():
    rng = np.random.default_rng(2)
    uL, uR = _states(rng, 40), _states(rng, 40)
    nt = rng.normal(size=(40, 2))
    H = ph.euler_roe(uL, uR, nt, G).v
    assert np.abs(H + ph.euler_roe(uR, uL, -nt, G).v).max() < 1e-12
    assert np.abs(2.5 * H - ph.euler_roe(uL, uR, 2.5 * nt, G).v).max() < 1e-12
    th = 0.7
    Rm = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    rot = lambda u: np.c_[u[:, 0], u[:, 1:3] @ Rm.T, u[:, 3]]
    Hr = ph.euler_roe(rot(uL), rot(uR), nt @ Rm.T, G).v
    assert np.abs(rot(H) - Hr).max() < 1e-12


def test_lf_burgers_closed_form_and_symmetry():
    rng = np.random.default_rng(3)
    uL, uR = rng.normal(size=(30, 1)), rng.normal(size=(30, 1))
    nt = rng.normal(size=(30, 2))
    H = ph.burgers_lf(uL, uR, nt).v[:, 0]
    a = np.maximum(np.abs(uL[:, 0] * nt[:, 0] + nt[:, 1]), np.abs(uR[:, 0] * nt[:, 0] + nt[:, 1]))
    fL = 0.5 * uL[:, 0] ** 2 * nt[:, 0] + uL[:, 0] * nt[:, 1]
    fR = 0.5 * uR[:, 0] ** 2 * nt[:, 0] + uR[:, 0] * nt[:, 1]
    assert np.abs(H - (0.5 * (fL + fR) - 0.5 * a * (uR[:, 0] - uL[:, 0]))).max() < 1e-15
    assert np.abs(H + ph.burgers_lf(uR, uL, -nt).v[:, 0]).max() < 1e-15
    assert np.abs(ph.burgers_lf(uL, uL, nt).v[:, 0] - fL).max() < 1e-15


@pytest.mark.parametrize("fix", [False, True])
def test_roe_dual_derivative_matches_fd(fix):
    rng = np.random.default_rng(4)
    k = 20
    uL, uR = _states(rng, k), _states(rng, k)
    if fix:  # near-sonic / near-stagnation faces exercise the entropy fix branch
        uR = uL * (1 + 0.05 * rng.normal(size=uL.shape))
        uR[:, 1:3] *= 0.01
        uL[:, 1:3] *= 0.01
    nt = rng.normal(size=(k, 2))
    x = np.c_[uL, uR, nt]
    d = Dual.seed(x, 0, 10)
    H = ph.euler_roe(d[:, 0:4], d[:, 4:8], d[:, 8:10], G)
    Jfd = np.zeros((k, 4, 10))
    for j in range(10):
        h = 1e-6 * max(1.0, np.abs(x[:, j]).max())
        xp, xm = x.copy(), x.copy()
        xp[:, j] += h
        xm[:, j] -= h
        Jfd[:, :, j] = (ph.euler_roe(xp[:, :4], xp[:, 4:8], xp[:, 8:], G).v
                        - ph.euler_roe(xm[:, :4], xm[:, 4:8], xm[:, 8:], G).v) / (2 * h)
    assert np.linalg.norm(H.d - Jfd) / np.linalg.norm(Jfd) < 1e-7


def test_wall_state_reflects_normal_momentum():
    u = np.array([[1.3, 0.4, 0.9, 3.0]])
    nt = np.array([[0.0, -2.0]])
    prm = {"gamma": G}
    ub = ph.boundary_state("euler", 3, u, nt, (2.0, 0.0), prm).v
    assert np.allclose(ub, [[1.3, 0.4, -0.9, 3.0]], atol=1e-15)
    fs = ph.euler_free_stream((2.0, 3.0), G)
    rho, vx, vy = fs[0], fs[1] / fs[0], fs[2] / fs[0]
    p = (G - 1) * (fs[3] - 0.5 * rho * (vx ** 2 + vy ** 2))
    assert abs(rho - 1) < 1e-15 and abs(p - 1) < 1e-14
    assert abs(np.hypot(vx, vy) - 2.0 * np.sqrt(G)) < 1e-14
    assert abs(np.degrees(np.arctan2(vy, vx)) - 3.0) < 1e-12


def test_roe_upwinds_a_single_contact_wave():
    """A density jump at equal velocity and pressure is one contact wave; with
    v.n above the entropy-fix threshold Roe's flux is the upwind flux f(uL).n~
    (and f(uR).n~ when v.n < 0)."""
    for sgn in (1.0, -1.0):
        v = sgn * np.array([1.5, 0.4])
        nt = np.array([[2.0, 0.0]])
        def st(rho):
            return np.array([[rho, rho * v[0], rho * v[1], 1.0 / (G - 1) + 0.5 * rho * v @ v]])
        uL, uR = st(1.0), st(2.3)
        H = ph.euler_roe(uL, uR, nt, G).v
        up = uL if sgn > 0 else uR
        assert np.abs(H - ph.euler_flux(up, G).v[0] @ nt[0]).max() < 1e-13


def test_lf_is_monotone():
    """dH/du- >= 0 >= dH/du+ (the local Lax-Friedrichs flux is an E-flux)."""
    rng = np.random.default_rng(9)
    x = np.c_[rng.normal(size=(200, 2)), rng.normal(size=(200, 2))]
    d = Dual.seed(x, 0, 4)
    H = ph.burgers_lf(d[:, 0:1], d[:, 1:2], d[:, 2:4])
    assert (H.d[:, 0, 0] >= -1e-15).all() and (H.d[:, 0, 1] <= 1e-15).all()


def test_harten_fix_is_c1_at_the_threshold():
    """Harten's fix replaces |lam| below delta by the parabola
    (lam^2 + delta^2) / (2 delta): it equals |lam| = delta with slope +-1 at
    |lam| = delta (C^1 joint), takes its minimum delta / 2 at lam = 0, and
    leaves |lam| >= delta untouched (Sec. 4.2 reading of the Roe flux)."""
    for delta in (0.07, 0.3, 1.9):
        d = Dual.seed(np.array([0.0]), 0, 1)
        dl = 0.0 * d + delta            # a constant Dual
        eps = 1e-9 * delta
        for sgn in (1.0, -1.0):
            lo = ph.harten_abs(d + sgn * (delta - eps), dl)
            hi = ph.harten_abs(d + sgn * (delta + eps), dl)
            # value continuity at the joint (a jump of O(delta) fails)
            assert abs(lo.v[0] - delta) < 1e-8 * delta
            assert abs(hi.v[0] - delta) < 1e-8 * delta
            # slope continuity: d/dlam = sign(lam) on both sides
            assert abs(lo.d[0, 0] - sgn) < 1e-8 and abs(hi.d[0, 0] - sgn) == 0.0
        mid = ph.harten_abs(d + 0.0, dl)
        assert abs(mid.v[0] - 0.5 * delta) < 1e-15 * delta and abs(mid.d[0, 0]) < 1e-15
        q = ph.harten_abs(d + 0.25 * delta, dl)
        # (1/16 + 1) delta^2 / (2 delta) = 17/32 delta, slope 1/4
        assert abs(q.v[0] - 17.0 / 32.0 * delta) < 1e-15 and abs(q.d[0, 0] - 0.25) < 1e-14


def _slow_contact_flux(rhoL, rhoR, v, p, nt):
    """Roe flux across a pure contact (equal velocity and pressure) written out
    by hand: only the entropy wave carries strength, alpha_2 = rho_R - rho_L
    along r_2 = (1, u, v, |v|^2 / 2), at speed v.n.  Its Roe-averaged sound
    speed has the closed form c~^2 = gamma p / sqrt(rho_L rho_R), and with
    |v.n| < delta = c~ / 10 the fixed speed is (vn^2 + delta^2) / (2 delta)."""
    nmag = np.hypot(*nt)
    n = nt / nmag
    vn = v @ n
    ct = np.sqrt(G * p / np.sqrt(rhoL * rhoR))
    delta = 0.1 * ct
    assert abs(vn) < delta
    lam_fix = (vn * vn + delta * delta) / (2.0 * delta)
    def fn(rho):
        E = p / (G - 1) + 0.5 * rho * (v @ v)
        m = rho * v
        return np.array([m @ nt, m[0] * (v @ nt) + p * nt[0], m[1] * (v @ nt) + p * nt[1], (E + p) * (v @ nt)])
    r2 = np.array([1.0, v[0], v[1], 0.5 * (v @ v)])
    return 0.5 * (fn(rhoL) + fn(rhoR)) - 0.5 * nmag * lam_fix * (rhoR - rhoL) * r2


def _contact_states(rhoL, rhoR, v, p):
    st = lambda rho: np.array([rho, rho * v[0], rho * v[1], p / (G - 1) + 0.5 * rho * (v @ v)])
    return st(rhoL)[None], st(rhoR)[None]


def test_roe_flux_at_a_slow_contact_matches_hand_computation():
    for v, nt in ((np.array([0.03, 0.2]), np.array([1.0, 0.0])),
                  (np.array([-0.02, 0.05]), np.array([0.6, -1.7])),
                  (np.array([0.0, 0.0]), np.array([0.0, 2.0]))):
        rhoL, rhoR, p = 1.0, 2.25, 1.3
        uL, uR = _contact_states(rhoL, rhoR, v, p)
        H = ph.euler_roe(uL, uR, nt[None], G).v[0]
        ref = _slow_contact_flux(rhoL, rhoR, v, p, nt)
        assert np.abs(H - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())
