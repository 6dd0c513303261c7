"""Seeded synthetic workloads shaped like the paper's two benchmarks.

Input generation only (no residual, flux, quadrature or solver arithmetic):
meshes, reduced bases Phi (state) and Psi (mapping), empirical-quadrature
(EQ) sets {(e_k, rho_k)}, parameters mu and reduced evaluation points.
Every generator is deterministic in its seed (NumPy PCG64).

Workloads
---------
``tiny_burgers``   P1 scalar problem with the space-time Burgers flux on an
                   8x8-cell mesh of [0,1]^2 (128 elements), n = 4, m = 3,
                   40 EQ elements.  Stands in for the shape of the paper's
                   Burgers benchmark (P1 simplices, scalar, space-time flux;
                   Section 4.1).
``spacetime_burgers``  the paper's space-time Burgers problem (Section 4.1)
                   on (0, 100) x (0, 50): source amplitude 0.02, inflow
                   u = mu[0] at x = 0 and u = 1 at t = 0, mu = (a, b) in
                   [3, 9] x [0.02, 0.075]; P1 or P2 on an nx x ny mesh.
``euler_p2``       P2 compressible Euler on a 128x64-cell mesh of [0,2]x[0,1]
                   (16384 elements), n = 20, m = 10, 819 EQ elements (5 %).
                   Stands in for the shape of the paper's NACA0012 benchmark
                   (P2 Euler, about 5 % non-zero EQ weights; Section 4.2).
                   Smaller meshes use the same recipe.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .mesh import Mesh, structured_mesh

GAMMA = 1.4


@dataclass
class Workload:
    name: str
    pde: str                  # "burgers" | "euler"
    p: int                    # DG degree (= mapping degree q)
    mesh: Mesh
    n_c: int                  # conservation-law components
    Phi: np.ndarray           # [N_u, n]
    Psi: np.ndarray           # [N_x, m]
    eq_elem: np.ndarray       # [n_s] int32, sorted, distinct
    eq_rho: np.ndarray        # [n_s] float64 > 0
    mus: np.ndarray           # [n_eval, n_mu]
    w_eval: np.ndarray        # [n_eval, n]
    tau_eval: np.ndarray      # [n_eval, m]
    kappa: float = 0.1
    eps_g: float = 1e-8
    gamma: float = GAMMA
    bc_mu_scale: float = 0.5  # Burgers inflow u_b = 1 + bc_mu_scale * mu[0]
    all_farfield: bool = False
    src_amp: float = 0.0      # Burgers source amplitude s_0 (s = s_0 exp(mu[1] x)); 0: none
    bc_spacetime: bool = False  # Burgers: u = mu[0] on the left edge, u = 1 on the bottom edge
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.Phi.shape[1]

    @property
    def m(self) -> int:
        return self.Psi.shape[1]

    @property
    def n_s(self) -> int:
        return self.eq_elem.shape[0]

    @property
    def X(self) -> np.ndarray:
        """Flattened reference coordinates [N_x] = [x0, y0, x1, y1, ...]."""
        return self.mesh.X.reshape(-1).copy()

    @property
    def n_nodes(self) -> int:
        return (self.p + 1) * (self.p + 2) // 2

    @property
    def N_u(self) -> int:
        return self.mesh.n_elem * self.n_nodes * self.n_c


def orthonormal_columns(A: np.ndarray) -> np.ndarray:
    """Q factor of a thin QR, signs fixed so that diag(R) > 0."""
    Q, R = np.linalg.qr(A)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def _rescale_l1(t: np.ndarray) -> np.ndarray:
    nrm = np.abs(t).sum()
    return t / max(1.0, nrm)


# ---------------------------------------------------------------- mapping modes
def _psi_from_modes(Xg: np.ndarray, modes, A: float) -> np.ndarray:
    """Raw (not orthonormalised) sinusoidal node displacements.

    Each mode is ("x", fx, fy) -> d = (A sin(fx X) cos(fy Y), 0) or
    ("y", fx, fy) -> d = (0, A cos(fx X) sin(fy Y)); the frequencies make
    d_x vanish on x = 0, Lx and d_y vanish on y = 0, Ly, so every boundary
    node slides tangentially along its boundary.
    """
    Xn, Yn = Xg[:, 0], Xg[:, 1]
    cols = []
    for kind, fx, fy in modes:
        d = np.zeros_like(Xg)
        if kind == "x":
            d[:, 0] = A * np.sin(fx * Xn) * np.cos(fy * Yn)
        else:
            d[:, 1] = A * np.cos(fx * Xn) * np.sin(fy * Yn)
        cols.append(d.reshape(-1))
    return np.stack(cols, axis=1)


def psi_tiny(mesh: Mesh, A: float = 0.05) -> np.ndarray:
    pi = np.pi
    modes = [("x", pi, pi), ("y", pi, pi), ("x", 2 * pi, pi)]
    return _psi_from_modes(mesh.X, modes, A)


EULER_PSI_PAIRS = [(1, 1), (1, 1), (2, 1), (1, 2), (1, 2), (2, 1), (2, 2), (2, 2), (3, 1), (1, 3)]


def psi_euler(mesh: Mesh, m: int, A: float = 0.05) -> np.ndarray:
    """Alternating x-type / y-type modes on [0, Lx] x [0, Ly]."""
    pi = np.pi
    modes = []
    for k in range(m):
        a, b = EULER_PSI_PAIRS[k % len(EULER_PSI_PAIRS)]
        shift = k // len(EULER_PSI_PAIRS)          # more modes: raise frequencies
        a, b = a + shift, b + shift
        if k % 2 == 0:
            modes.append(("x", pi * a / mesh.Lx, pi * b / mesh.Ly))
        else:
            modes.append(("y", pi * a / mesh.Lx, pi * b / mesh.Ly))
    return _psi_from_modes(mesh.X, modes, A)


# --------------------------------------------------------------- state fields
def euler_reference_state(mesh: Mesh, M: float = 2.5, gamma: float = GAMMA,
                          width: float = 0.03, ratio: float = 2.5) -> np.ndarray:
    """Free stream with a tanh jump of density and pressure across the line
    x = 0.6 + 0.4 y (ratio ``ratio``), velocity unchanged.  Sampled at every
    element node; returns U_ref [N_u] in element-major layout."""
    xy = mesh.node_coords()                         # [Ne, nn, 2]
    s = (xy[..., 0] - 0.4 * xy[..., 1] - 0.6) / np.sqrt(1.0 + 0.16)
    H = 0.5 * (1.0 + np.tanh(s / width))
    fac = 1.0 + (ratio - 1.0) * H
    v = M * np.sqrt(gamma)
    rho = fac
    p = fac
    U = np.stack([rho, rho * v, 0.0 * rho, p / (gamma - 1.0) + 0.5 * rho * v * v], axis=-1)
    return U.reshape(-1)


def smooth_field(mesh: Mesh, rng: np.random.Generator, n_c: int, K: int = 8) -> np.ndarray:
    """Sum_{a,b<K} c_ab exp(-(a^2+b^2)/8) cos(pi a X / Lx + th) cos(pi b Y / Ly + th'),
    drawn independently per component and sampled at the element nodes."""
    xy = mesh.node_coords()
    Xn = xy[..., 0] / mesh.Lx
    Yn = xy[..., 1] / mesh.Ly
    out = np.zeros(xy.shape[:2] + (n_c,))
    a = np.arange(K)
    ax = np.pi * a[None, :] * Xn.reshape(-1, 1)          # [P, K]
    by = np.pi * a[None, :] * Yn.reshape(-1, 1)
    cx, sx, cy, sy = np.cos(ax), np.sin(ax), np.cos(by), np.sin(by)
    for c in range(n_c):
        coef = rng.standard_normal((K, K)) * np.exp(-(a[:, None] ** 2 + a[None, :] ** 2) / 8.0)
        th = rng.uniform(0, 2 * np.pi, (K, K))
        th2 = rng.uniform(0, 2 * np.pi, (K, K))
        # cos(A + th) cos(B + th') expanded so the double sum separates in (a, b)
        val = np.zeros(Xn.size)
        for fa, ga in ((cx, np.cos(th)), (sx, -np.sin(th))):
            for fb, gb in ((cy, np.cos(th2)), (sy, -np.sin(th2))):
                val += np.einsum("pb,pb->p", fa @ (coef * ga * gb), fb)
        out[..., c] = val.reshape(Xn.shape)
    return out.reshape(-1)


# ------------------------------------------------------------------ workloads
def tiny_burgers(n_eval: int = 16, nx: int = 8, ny: int = 8, n: int = 4, n_s: int = 40,
                 kappa: float = 0.1) -> Workload:
    mesh = structured_mesh(nx, ny, 1.0, 1.0, 1)
    N_u = mesh.n_elem * 3
    Phi = orthonormal_columns(np.random.default_rng(1001).standard_normal((N_u, n)))
    Psi = psi_tiny(mesh)
    rng = np.random.default_rng(1003)
    eq_elem = np.sort(rng.choice(mesh.n_elem, size=min(n_s, mesh.n_elem), replace=False)).astype(np.int32)
    eq_rho = rng.uniform(0.5, 2.0, size=eq_elem.shape[0])
    rng = np.random.default_rng(1004)
    m = Psi.shape[1]
    w = np.sqrt(N_u / n) * rng.standard_normal((n_eval, n))
    tau = np.stack([_rescale_l1(rng.uniform(-1, 1, m)) for _ in range(n_eval)])
    mus = np.full((n_eval, 1), 0.3)
    return Workload("tiny_burgers", "burgers", 1, mesh, 1, Phi, Psi, eq_elem, eq_rho,
                    mus, w, tau, kappa=kappa)


def spacetime_burgers(n_eval: int = 16, nx: int = 8, ny: int = 8, p: int = 1, n: int = 4, m: int = 4,
                      n_s: int = 40, kappa: float = 0.1) -> Workload:
    """Space-time Burgers on (0, 100) x (0, 50) with the paper's source and
    initial/boundary data; mapping modes as for the Euler workload, with
    amplitude 5 % of the domain height."""
    mesh = structured_mesh(nx, ny, 100.0, 50.0, p)
    nn = (p + 1) * (p + 2) // 2
    N_u = mesh.n_elem * nn
    Phi = orthonormal_columns(np.random.default_rng(1001).standard_normal((N_u, n)))
    Psi = psi_euler(mesh, m, A=2.5)
    rng = np.random.default_rng(1003)
    eq_elem = np.sort(rng.choice(mesh.n_elem, size=min(n_s, mesh.n_elem), replace=False)).astype(np.int32)
    eq_rho = rng.uniform(0.5, 2.0, size=eq_elem.shape[0])
    rng = np.random.default_rng(1004)
    w = np.sqrt(N_u / n) * rng.standard_normal((n_eval, n))
    tau = np.stack([_rescale_l1(rng.uniform(-1, 1, m)) for _ in range(n_eval)])
    mus = np.stack([rng.uniform(3.0, 9.0, n_eval), rng.uniform(0.02, 0.075, n_eval)], axis=1)
    return Workload(f"spacetime_burgers_p{p}", "burgers", p, mesh, 1, Phi, Psi, eq_elem, eq_rho,
                    mus, w, tau, kappa=kappa, src_amp=0.02, bc_spacetime=True)


def euler_p2(nx: int = 128, ny: int = 64, n: int = 20, m: int = 10, n_s: int | None = None,
             n_eval: int = 16, seed_phi: int = 1001, kappa: float = 0.1,
             alpha_deg: float = 0.0, all_farfield: bool = False,
             rho_dist: str = "lognormal", p: int = 2) -> Workload:
    """The Euler workload; P2 (the benchmark) unless p = 1."""
    mesh = structured_mesh(nx, ny, 2.0, 1.0, p)
    if n_s is None:
        n_s = max(1, int(round(0.05 * mesh.n_elem)))
    U_ref = euler_reference_state(mesh)
    N_u = U_ref.shape[0]
    cols = []
    for c in range(4):
        e = np.zeros(N_u)
        e[c::4] = 1.0
        cols.append(e)
    cols.append(U_ref)
    rng = np.random.default_rng(seed_phi)
    for _ in range(max(0, n - 5)):
        cols.append(smooth_field(mesh, rng, 4))
    Phi = orthonormal_columns(np.stack(cols[:n], axis=1))
    Psi = psi_euler(mesh, m)
    rng = np.random.default_rng(1003)
    eq_elem = np.sort(rng.choice(mesh.n_elem, size=min(n_s, mesh.n_elem), replace=False)).astype(np.int32)
    if rho_dist == "lognormal":
        eq_rho = rng.lognormal(0.0, 0.5, size=eq_elem.shape[0])
    else:
        eq_rho = np.ones(eq_elem.shape[0])
    rng = np.random.default_rng(1004)
    mach = rng.uniform(2.0, 3.0, n_eval)
    mus = np.stack([mach, np.full(n_eval, alpha_deg)], axis=1)
    w0 = Phi.T @ U_ref
    scale = 0.02 * np.linalg.norm(U_ref) / np.sqrt(n)
    w = w0[None, :] + scale * rng.standard_normal((n_eval, n))
    tau = np.stack([_rescale_l1(rng.uniform(-1, 1, m)) for _ in range(n_eval)])
    return Workload(f"euler_p{p}", "euler", p, mesh, 4, Phi, Psi, eq_elem, eq_rho, mus, w, tau,
                    kappa=kappa, all_farfield=all_farfield, extra={"U_ref": U_ref})


def with_eq(wl: Workload, eq_elem: np.ndarray, eq_rho: np.ndarray) -> Workload:
    """Same workload with another EQ set (e.g. all elements with rho = 1)."""
    import copy
    out = copy.copy(wl)
    out.eq_elem = np.asarray(eq_elem, dtype=np.int32)
    out.eq_rho = np.asarray(eq_rho, dtype=np.float64)
    return out


def inflow_elements(mesh: Mesh) -> np.ndarray:
    """Elements with a face on the inflow boundary (tag 1, x = 0)."""
    return np.nonzero((mesh.elem_nbr == -1).any(axis=1))[0].astype(np.int32)


def eq_set_with_inflow(mesh: Mesh, n_random: int, rng: np.random.Generator) -> np.ndarray:
    """Sorted EQ element set: n_random elements drawn without replacement,
    joined with every inflow-boundary element.  Near a uniform state a
    uniform change of the state is seen only by inflow elements, so a
    sampled set without them leaves the constant directions of the reduced
    basis undetermined; any trained EQ rule contains such elements."""
    inflow = inflow_elements(mesh)
    rest = np.setdiff1d(np.arange(mesh.n_elem), inflow)
    pick = rng.choice(rest, size=min(n_random, rest.size), replace=False)
    return np.sort(np.concatenate([inflow, pick])).astype(np.int32)


@dataclass
class BatchWorkload:
    """Many ROM instances on one mesh: a pool of bases and, per instance,
    the pool index, its EQ set and weights, and mu = (Mach, angle in deg)."""
    mesh: Mesh
    pool: list            # [(Phi, Psi)] bases of the pool ROMs
    pool_nm: list         # [(n, m)]
    inst_pool: np.ndarray
    inst_elem: list
    inst_rho: list
    mus: np.ndarray       # [n_inst, 2]
    base: Workload        # the workload whose mesh and constants the pool shares


def euler_batch(n_inst: int = 1024, nx: int = 128, ny: int = 64, ns_lo: int = 200, ns_hi: int = 2000,
                ns_list=None) -> BatchWorkload:
    """Batched instances of the P2 Euler workload: pool of 6 ROMs with
    n in {10, 20, 30} x m in {5, 10} (pool entry p built like the single
    workload with basis seed 1001 + p), mu from a scrambled Sobol sequence
    (seed 1005) on [2, 3] x [-5, 5] degrees, pool index per instance
    uniform (seed 1008), EQ set sizes U{ns_lo..ns_hi} (or ns_list) drawn
    (seed 1009) with the inflow elements added, weights lognormal(0, 0.5)."""
    from scipy.stats import qmc
    pool_nm = [(n, m) for n in (10, 20, 30) for m in (5, 10)]
    base = euler_p2(nx=nx, ny=ny, n=30, m=10, n_s=1, n_eval=1)
    mesh = base.mesh
    U_ref = base.extra["U_ref"]
    pool = []
    for p, (n, m) in enumerate(pool_nm):
        N_u = U_ref.shape[0]
        cols = []
        for c in range(4):
            e = np.zeros(N_u)
            e[c::4] = 1.0
            cols.append(e)
        cols.append(U_ref)
        rng = np.random.default_rng(1001 + p)
        for _ in range(max(0, n - 5)):
            cols.append(smooth_field(mesh, rng, 4))
        pool.append((orthonormal_columns(np.stack(cols[:n], axis=1)), psi_euler(mesh, m)))
    sob = qmc.Sobol(d=2, scramble=True, seed=1005).random(n_inst)
    mus = np.stack([2.0 + sob[:, 0], -5.0 + 10.0 * sob[:, 1]], axis=1)
    inst_pool = np.random.default_rng(1008).integers(0, len(pool), n_inst)
    rng = np.random.default_rng(1009)
    sizes = (np.asarray(ns_list) if ns_list is not None else rng.integers(ns_lo, ns_hi + 1, n_inst))
    inst_elem, inst_rho = [], []
    for i in range(n_inst):
        el = eq_set_with_inflow(mesh, int(sizes[i % len(sizes)]), rng)
        inst_elem.append(el)
        inst_rho.append(rng.lognormal(0.0, 0.5, size=el.size))
    return BatchWorkload(mesh, pool, pool_nm, inst_pool, inst_elem, inst_rho, mus, base)
