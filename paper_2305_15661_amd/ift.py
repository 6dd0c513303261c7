"""Thin ctypes binding of the C ABI in include/ift.h (argument marshalling only).

Every function here forwards to ``libift.so``; all element, reduction and
solver arithmetic runs in the library's HIP kernels.  Device arrays are
torch tensors on the current CUDA/HIP device (float64, contiguous); the
stream is torch's current stream unless one is given.  If the library has
not been built this module raises at first use instead of falling back to
any CPU path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libift.so")

IFT_OK, IFT_EINVAL, IFT_ENOMEM, IFT_EDEVICE = 0, -1, -2, -3
IFT_EBADMESH, IFT_ENONPHYS, IFT_ESINGULAR, IFT_ELINESEARCH, IFT_ENOTCONV = -4, -5, -6, -7, -8
IFT_ESCRATCH = -9
NOALLOC_SCRATCH_BYTES = 32 << 20   # IFT_NOALLOC_SCRATCH_BYTES of include/ift.h
STATUS_NAMES = {0: "IFT_OK", -1: "IFT_EINVAL", -2: "IFT_ENOMEM", -3: "IFT_EDEVICE", -4: "IFT_EBADMESH",
                -5: "IFT_ENONPHYS", -6: "IFT_ESINGULAR", -7: "IFT_ELINESEARCH", -8: "IFT_ENOTCONV",
                -9: "IFT_ESCRATCH"}
PDE = {"burgers": 0, "euler": 1}
PRECISION = {"fp64": 0, "fp32": 1, "mixed": 2}


class IftError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}")
        self.status = status


class ProblemDesc(ctypes.Structure):
    _fields_ = [("pde", ctypes.c_int), ("p", ctypes.c_int), ("n_elem", ctypes.c_int), ("n_gnode", ctypes.c_int),
                ("X", ctypes.POINTER(ctypes.c_double)), ("elem_gnodes", ctypes.POINTER(ctypes.c_int)),
                ("elem_nbr", ctypes.POINTER(ctypes.c_int)), ("gamma", ctypes.c_double), ("kappa", ctypes.c_double),
                ("eps_g", ctypes.c_double), ("bc_mu_scale", ctypes.c_double), ("all_farfield", ctypes.c_int),
                ("src_amp", ctypes.c_double), ("bc_spacetime", ctypes.c_int)]


class GNParams(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("c1", ctypes.c_double), ("max_backtrack", ctypes.c_int),
                ("tol", ctypes.c_double), ("tol_mix", ctypes.c_double), ("max_backtrack_mixed", ctypes.c_int),
                ("use_qr", ctypes.c_int), ("w_only", ctypes.c_int)]


class GNInfo(ctypes.Structure):
    _fields_ = [("J_old", ctypes.c_double), ("J_new", ctypes.c_double), ("alpha", ctypes.c_double),
                ("norm_S", ctypes.c_double), ("norm_T", ctypes.c_double), ("n_backtrack", ctypes.c_int),
                ("converged", ctypes.c_int), ("status", ctypes.c_int), ("iterations", ctypes.c_int),
                ("fallback", ctypes.c_int), ("mixed_iterations", ctypes.c_int),
                ("presolve_iterations", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
EXPORTS = {
    "ift_problem_create": (ctypes.c_int, [ctypes.POINTER(ProblemDesc), ctypes.POINTER(_P)]),
    "ift_problem_destroy": (None, [_P]),
    "ift_problem_sizes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_longlong),
                                         ctypes.POINTER(ctypes.c_longlong)]),
    "ift_problem_neighbour_map": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_longlong)]),
    "hdm_assemble": (ctypes.c_int, [_P, _D, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "eq_element_contributions": (ctypes.c_int, [_P, _D, _P, _P, _P, _P]),
    "hdm_residual_norm_batched": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_int, _P, _P, ctypes.c_int, _P,
                                                 _P, _P, _P]),
    "ift_rom_create": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, _P, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int), _D, ctypes.c_int, ctypes.POINTER(_P)]),
    "ift_rom_destroy": (None, [_P]),
    "ift_rom_get_gathers": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "eq_assemble_residual": (ctypes.c_int, [_P, _D, _P, _P, _P, _P, _P, _P, _P]),
    "eq_assemble_jacobian": (ctypes.c_int, [_P, _D, _P, _P, _P, _P, _P, _P, _P, _P]),
    "eq_assemble_jacobian_noalloc": (ctypes.c_int, [_P, _D, _P, _P, _P, _P, _P, _P, _P]),
    "eq_noalloc_scratch_bytes": (ctypes.c_size_t, [_P]),
    "rom_gauss_newton_step": (ctypes.c_int, [_P, _D, _P, _P, ctypes.POINTER(GNParams), ctypes.POINTER(GNInfo), _P]),
    "ift_rom_reserve": (ctypes.c_int, [_P, ctypes.c_int]),
    "eq_assemble_residual_batch": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P, _P, _P]),
    "eq_assemble_jacobian_batch": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P, _P, _P, _P, _P]),
    "ift_batch_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(_P)]),
    "ift_batch_destroy": (None, [_P]),
    "ift_batch_layout": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "ift_batch_autotune": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(ctypes.c_int), _P]),
    "eq_assemble_jacobian_batched": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "rom_gauss_newton_solve_batched": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(GNParams), ctypes.c_int, _P,
                                                      ctypes.c_int, _P]),
    "rom_plain_start": (ctypes.c_int, [_P, _D, _P, _P, _P]),
    "rom_plain_start_batched": (ctypes.c_int, [_P, _P, _P, _P]),
    "ift_mlp_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_ulonglong,
                                      ctypes.POINTER(_P)]),
    "ift_mlp_destroy": (None, [_P]),
    "ift_mlp_num_params": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int)]),
    "ift_mlp_set_params": (ctypes.c_int, [_P, _P, _P]),
    "ift_mlp_get_params": (ctypes.c_int, [_P, _P, _P]),
    "ift_mlp_set_normalization": (ctypes.c_int, [_P, _D, _D, _D, _D]),
    "ift_mlp_loss_grad": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P, ctypes.POINTER(ctypes.c_double), _P]),
    "ift_mlp_train": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_double, _D, _P]),
    "ift_mlp_predict": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, ctypes.c_int, _P]),
    "ift_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "ift_profile_reset": (ctypes.c_int, []),
    "ift_profile_read": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]),
}
PROF = {"hdm": 0, "eq_res": 1, "eq_jac": 2, "gram": 3, "points": 4}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2305_15661_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(st: int, where: str):
    if st != IFT_OK:
        raise IftError(st, where)


def _ptr(t, n=None, dtype=None):
    """Device pointer of a contiguous torch tensor (or None)."""
    if t is None:
        return None
    import torch
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _mu(mu):
    a = (ctypes.c_double * 2)()
    mu = np.atleast_1d(np.asarray(mu, dtype=np.float64))
    for i in range(min(2, mu.size)):
        a[i] = mu[i]
    return a


class Problem:
    def __init__(self, pde: str, p: int, X, elem_gnodes, elem_nbr, gamma=1.4, kappa=0.1, eps_g=1e-8,
                 bc_mu_scale=0.5, all_farfield=False, src_amp=0.0, bc_spacetime=False):
        L = lib()
        self._X = np.ascontiguousarray(np.asarray(X, dtype=np.float64).reshape(-1))
        self._gn = np.ascontiguousarray(elem_gnodes, dtype=np.int32)
        self._nb = np.ascontiguousarray(elem_nbr, dtype=np.int32)
        d = ProblemDesc(PDE[pde], int(p), int(self._gn.shape[0]), int(self._X.size // 2),
                        self._X.ctypes.data_as(_D), self._gn.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                        self._nb.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), float(gamma), float(kappa),
                        float(eps_g), float(bc_mu_scale), int(bool(all_farfield)), float(src_amp),
                        int(bool(bc_spacetime)))
        h = _P()
        _check(L.ift_problem_create(ctypes.byref(d), ctypes.byref(h)), "ift_problem_create")
        self.handle = h
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        nu, nx = ctypes.c_longlong(), ctypes.c_longlong()
        _check(L.ift_problem_sizes(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(nu),
                                   ctypes.byref(nx)), "ift_problem_sizes")
        self.nue, self.nun, self.nxe, self.N_u, self.N_x = a.value, b.value, c.value, nu.value, nx.value
        self.n_elem = int(self._gn.shape[0])
        self.pde = pde

    @classmethod
    def from_workload(cls, wl):
        return cls(wl.pde, wl.p, wl.mesh.X, wl.mesh.elem_gnodes, wl.mesh.elem_nbr, gamma=wl.gamma,
                   kappa=wl.kappa, eps_g=wl.eps_g, bc_mu_scale=wl.bc_mu_scale, all_farfield=wl.all_farfield,
                   src_amp=getattr(wl, "src_amp", 0.0), bc_spacetime=getattr(wl, "bc_spacetime", False))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.ift_problem_destroy(h)
            self.handle = None

    def neighbour_map(self) -> np.ndarray:
        """ift_problem_neighbour_map: [n_elem][nun] indices into U, -1 on boundary faces."""
        out = np.zeros(self.n_elem * self.nun, dtype=np.int64)
        _check(lib().ift_problem_neighbour_map(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong))),
               "ift_problem_neighbour_map")
        return out.reshape(self.n_elem, self.nun)

    def hdm_assemble(self, mu, U, x, R=None, N=None, dRdU=None, dRdUn=None, dRdx=None, dNdx=None, n_bad=None,
                     stream=None):
        import torch
        f64 = torch.float64
        Ne, nue, nun, nxe = self.n_elem, self.nue, self.nun, self.nxe
        st = lib().hdm_assemble(self.handle, _mu(mu), _ptr(U, self.N_u, f64), _ptr(x, self.N_x, f64),
                                _ptr(R, self.N_u, f64), _ptr(N, Ne, f64), _ptr(dRdU, Ne * nue * nue, f64),
                                _ptr(dRdUn, Ne * nue * nun, f64), _ptr(dRdx, Ne * nue * nxe, f64),
                                _ptr(dNdx, Ne * nxe, f64), _ptr(n_bad, 1, torch.int32), _stream(stream))
        _check(st, "hdm_assemble")

    def hdm_residual_norms(self, mu, Phi, w, Psi, tau, norms, n_bad=None, stream=None):
        """hdm_residual_norm_batched: |R(Phi w_p; X + Psi tau_p, mu_p)|_2 for
        each row p of mu [P,2], w [P,n], tau [P,m] (device tensors), with the
        full bases Phi [N_u,n], Psi [N_x,m]; norms [P], n_bad [P] (int32)."""
        import torch
        f64 = torch.float64
        P, n = w.shape
        m = Psi.shape[1] if Psi is not None else 0
        st = lib().hdm_residual_norm_batched(self.handle, int(P), _ptr(mu, 2 * P, f64), _ptr(Phi, self.N_u * n, f64),
                                             int(n), _ptr(w, P * n, f64), _ptr(Psi, self.N_x * m, f64), int(m),
                                             _ptr(tau, P * m, f64), _ptr(norms, P, f64),
                                             _ptr(n_bad, P, torch.int32), _stream(stream))
        _check(st, "hdm_residual_norm_batched")


def greedy_select(norms) -> int:
    """Index of the candidate with the largest full-order residual norm, the
    next training parameter of eq. (greedy0) (host-side argmax).  A
    non-finite norm (the lifted state of that reduced solution is invalid)
    ranks above every finite one; ties go to the lowest index."""
    v = np.asarray(norms.cpu().numpy() if hasattr(norms, "cpu") else norms, dtype=np.float64)
    v = np.where(np.isfinite(v), v, np.inf)
    return int(np.argmax(v))


class ROM:
    def __init__(self, prob: Problem, Phi, Psi, eq_elem, eq_rho, precision="fp64"):
        import torch
        self.prob = prob
        self.n = int(Phi.shape[1])
        self.m = int(Psi.shape[1])
        self.D = self.n + self.m
        el = np.ascontiguousarray(eq_elem, dtype=np.int32)
        rho = np.ascontiguousarray(eq_rho, dtype=np.float64)
        if rho.size != el.size:
            raise ValueError(f"{el.size} EQ elements but {rho.size} weights")
        self.n_s = int(el.size)
        h = _P()
        st = lib().ift_rom_create(prob.handle, self.n, self.m, _ptr(Phi, prob.N_u * self.n, torch.float64),
                                  _ptr(Psi, prob.N_x * self.m, torch.float64) if self.m else None, self.n_s,
                                  el.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), rho.ctypes.data_as(_D),
                                  PRECISION[precision], ctypes.byref(h))
        _check(st, "ift_rom_create")
        self.handle = h
        self.nrows = self.n_s * prob.nue + self.n_s

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.ift_rom_destroy(h)
            self.handle = None

    def get_gathers(self, Phi_s=None, Phin_s=None, Psi_s=None, X_s=None, stream=None):
        import torch
        f64, p = torch.float64, self.prob
        _check(lib().ift_rom_get_gathers(self.handle, _ptr(Phi_s, self.n_s * p.nue * self.n, f64),
                                         _ptr(Phin_s, self.n_s * p.nun * self.n, f64),
                                         _ptr(Psi_s, self.n_s * p.nxe * self.m, f64),
                                         _ptr(X_s, self.n_s * p.nxe, f64), _stream(stream)), "ift_rom_get_gathers")

    def eq_assemble_residual(self, mu, w, tau, Jobj, Ft=None, PhiT_r=None, n_bad=None, stream=None):
        import torch
        f64 = torch.float64
        st = lib().eq_assemble_residual(self.handle, _mu(mu), _ptr(w, self.n, f64), _ptr(tau, self.m, f64),
                                        _ptr(Jobj, 1, f64), _ptr(Ft, self.nrows, f64), _ptr(PhiT_r, self.n, f64),
                                        _ptr(n_bad, 1, torch.int32), _stream(stream))
        _check(st, "eq_assemble_residual")

    def eq_assemble_jacobian(self, mu, w, tau, Jobj, g, H, Jt=None, n_bad=None, stream=None):
        import torch
        f64 = torch.float64
        st = lib().eq_assemble_jacobian(self.handle, _mu(mu), _ptr(w, self.n, f64), _ptr(tau, self.m, f64),
                                        _ptr(Jobj, 1, f64), _ptr(g, self.D, f64), _ptr(H, self.D * self.D, f64),
                                        _ptr(Jt, self.nrows * self.D, f64), _ptr(n_bad, 1, torch.int32),
                                        _stream(stream))
        _check(st, "eq_assemble_jacobian")

    def eq_assemble_jacobian_noalloc(self, mu, w, tau, Jobj, g, H, n_bad=None, stream=None):
        """eq_assemble_jacobian_noalloc: the same outputs (no Jt) with the
        library's static device scratch instead of allocated workspaces."""
        import torch
        f64 = torch.float64
        st = lib().eq_assemble_jacobian_noalloc(self.handle, _mu(mu), _ptr(w, self.n, f64), _ptr(tau, self.m, f64),
                                                _ptr(Jobj, 1, f64), _ptr(g, self.D, f64),
                                                _ptr(H, self.D * self.D, f64), _ptr(n_bad, 1, torch.int32),
                                                _stream(stream))
        _check(st, "eq_assemble_jacobian_noalloc")

    def noalloc_scratch_bytes(self):
        return int(lib().eq_noalloc_scratch_bytes(self.handle))

    def element_contributions(self, mu, w, tau, C, stream=None):
        """eq_element_contributions: C [n_s, n+m] device tensor of the
        unweighted elemental reduced residuals at (mu, w, tau)."""
        import torch
        f64 = torch.float64
        st = lib().eq_element_contributions(self.handle, _mu(mu), _ptr(w, self.n, f64), _ptr(tau, self.m, f64),
                                            _ptr(C, self.n_s * self.D, f64), _stream(stream))
        _check(st, "eq_element_contributions")

    def reserve(self, max_pts: int):
        _check(lib().ift_rom_reserve(self.handle, int(max_pts)), "ift_rom_reserve")

    def eq_assemble_residual_batch(self, mu, w, tau, Jobj, n_bad=None, stream=None):
        """mu [P,2], w [P,n], tau [P,m] device tensors; Jobj [P]."""
        import torch
        f64 = torch.float64
        P = int(w.shape[0])
        st = lib().eq_assemble_residual_batch(self.handle, P, _ptr(mu, 2 * P, f64), _ptr(w, P * self.n, f64),
                                              _ptr(tau, P * self.m, f64), _ptr(Jobj, P, f64),
                                              _ptr(n_bad, P, torch.int32), _stream(stream))
        _check(st, "eq_assemble_residual_batch")

    def eq_assemble_jacobian_batch(self, mu, w, tau, Jobj, g, H, n_bad=None, stream=None):
        """mu [P,2], w [P,n], tau [P,m]; Jobj [P], g [P,D], H [P,D,D] device tensors."""
        import torch
        f64 = torch.float64
        P = int(w.shape[0])
        st = lib().eq_assemble_jacobian_batch(self.handle, P, _ptr(mu, 2 * P, f64), _ptr(w, P * self.n, f64),
                                              _ptr(tau, P * self.m, f64), _ptr(Jobj, P, f64),
                                              _ptr(g, P * self.D, f64), _ptr(H, P * self.D * self.D, f64),
                                              _ptr(n_bad, P, torch.int32), _stream(stream))
        _check(st, "eq_assemble_jacobian_batch")

    def plain_start(self, mu, w, tau, stream=None):
        """w = Phi^T U_fs(mu), tau = 0 (device tensors, overwritten)."""
        import torch
        f64 = torch.float64
        _check(lib().rom_plain_start(self.handle, _mu(mu), _ptr(w, self.n, f64), _ptr(tau, self.m, f64),
                                     _stream(stream)), "rom_plain_start")

    def gauss_newton_step(self, mu, w, tau, lam=0.0, c1=1e-4, max_backtrack=30, tol=1e-8, qr=False, w_only=False,
                          stream=None):
        """rom_gauss_newton_step; returns (status, info dict).  Soft outcomes
        (converged / line-search failure / invalid point) are reported in the
        status instead of raising.  qr: solve the step by Householder QR of
        the stacked rows instead of the normal equations; w_only: step in w
        with tau held, converged on |S~| alone."""
        import torch
        f64 = torch.float64
        prm = GNParams(float(lam), float(c1), int(max_backtrack), float(tol), 0.0, 0, int(bool(qr)),
                       int(bool(w_only)))
        info = GNInfo()
        st = lib().rom_gauss_newton_step(self.handle, _mu(mu), _ptr(w, self.n, f64), _ptr(tau, self.m, f64),
                                         ctypes.byref(prm), ctypes.byref(info), _stream(stream))
        if st in (IFT_EINVAL, IFT_ENOMEM, IFT_EDEVICE):
            raise IftError(st, "rom_gauss_newton_step")
        return st, info.as_dict()


# numpy view of a device array of ift_gn_info records
GN_INFO_DTYPE = np.dtype([("J_old", "<f8"), ("J_new", "<f8"), ("alpha", "<f8"), ("norm_S", "<f8"),
                          ("norm_T", "<f8"), ("n_backtrack", "<i4"), ("converged", "<i4"), ("status", "<i4"),
                          ("iterations", "<i4"), ("fallback", "<i4"), ("mixed_iterations", "<i4"),
                          ("presolve_iterations", "<i4"), ("_pad", "<i4")])
assert GN_INFO_DTYPE.itemsize == ctypes.sizeof(GNInfo)


class Batch:
    """Many ROM instances solved together (ift_batch_*).  The ROM objects
    must stay alive as long as the batch."""

    def __init__(self, roms):
        self.roms = list(roms)
        self.n_inst = len(self.roms)
        arr = (_P * self.n_inst)(*[r.handle for r in self.roms])
        h = _P()
        _check(lib().ift_batch_create(self.n_inst, arr, ctypes.byref(h)), "ift_batch_create")
        self.handle = h
        zo = (ctypes.c_int * (self.n_inst + 1))()
        ho = (ctypes.c_int * (self.n_inst + 1))()
        _check(lib().ift_batch_layout(h, zo, ho), "ift_batch_layout")
        self.zoff = np.array(zo[:], dtype=np.int64)
        self.hoff = np.array(ho[:], dtype=np.int64)
        self.nz = int(self.zoff[-1])
        self.nh = int(self.hoff[-1])

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.ift_batch_destroy(h)
            self.handle = None

    def pack(self, zs, device=None):
        """Packed device vector from a list of per-instance coordinate vectors."""
        import torch
        return torch.tensor(np.concatenate([np.asarray(z, dtype=np.float64) for z in zs]), dtype=torch.float64,
                            device=device or "cuda")

    def unpack(self, z):
        zz = z.detach().cpu().numpy() if hasattr(z, "detach") else np.asarray(z)
        return [zz[self.zoff[i]:self.zoff[i + 1]] for i in range(self.n_inst)]

    def plain_start(self, mu, z, stream=None):
        """Packed plain starts of every instance into z (device)."""
        import torch
        f64 = torch.float64
        _check(lib().rom_plain_start_batched(self.handle, _ptr(mu, 2 * self.n_inst, f64), _ptr(z, self.nz, f64),
                                             _stream(stream)), "rom_plain_start_batched")

    def autotune(self, mu, z, stream=None) -> int:
        import torch
        f64 = torch.float64
        c = ctypes.c_int()
        _check(lib().ift_batch_autotune(self.handle, _ptr(mu, 2 * self.n_inst, f64), _ptr(z, self.nz, f64),
                                        ctypes.byref(c), _stream(stream)), "ift_batch_autotune")
        return c.value

    def eq_assemble_jacobian(self, mu, z, Jobj, g, H, n_bad=None, stream=None):
        import torch
        f64 = torch.float64
        st = lib().eq_assemble_jacobian_batched(self.handle, _ptr(mu, 2 * self.n_inst, f64), _ptr(z, self.nz, f64),
                                                _ptr(Jobj, self.n_inst, f64), _ptr(g, self.nz, f64),
                                                _ptr(H, self.nh, f64), _ptr(n_bad, self.n_inst, torch.int32),
                                                _stream(stream))
        _check(st, "eq_assemble_jacobian_batched")

    def solve(self, mu, z, info, lam=0.0, c1=1e-4, max_backtrack=30, tol=1e-8, max_it=50, graph=True,
              warm=False, tol_mix=0.0, max_backtrack_mixed=0, presolve=False, adaptive_lambda=False, stream=None):
        """rom_gauss_newton_solve_batched; info: device uint8 tensor of
        n_inst * GN_INFO_DTYPE.itemsize bytes (see info_array).  tol_mix and
        max_backtrack_mixed (0: the library's defaults) steer the switch of
        mixed-precision instances to FP64 rounds."""
        import torch
        prm = GNParams(float(lam), float(c1), int(max_backtrack), float(tol), float(tol_mix),
                       int(max_backtrack_mixed))
        if info.numel() * info.element_size() != self.n_inst * GN_INFO_DTYPE.itemsize:
            raise ValueError("info has the wrong size")
        st = lib().rom_gauss_newton_solve_batched(self.handle, _ptr(mu, 2 * self.n_inst, torch.float64),
                                                  _ptr(z, self.nz, torch.float64), ctypes.byref(prm), int(max_it),
                                                  ctypes.c_void_p(info.data_ptr()),
                                                  (0 if graph else 1) | (2 if warm else 0) | (4 if presolve else 0)
                                                  | (8 if adaptive_lambda else 0), _stream(stream))
        _check(st, "rom_gauss_newton_solve_batched")

    def info_buffer(self, device=None):
        import torch
        return torch.zeros(self.n_inst * GN_INFO_DTYPE.itemsize, dtype=torch.uint8, device=device or "cuda")

    @staticmethod
    def info_array(buf):
        return np.frombuffer(buf.cpu().numpy().tobytes(), dtype=GN_INFO_DTYPE)


class MLP:
    """Warm-start network (ift_mlp_*): n_in -> hidden -> hidden -> n_out, GELU."""

    def __init__(self, n_in=2, hidden=128, n_out=30, seed=1):
        h = _P()
        _check(lib().ift_mlp_create(int(n_in), int(hidden), int(n_out), int(seed), ctypes.byref(h)), "ift_mlp_create")
        self.handle = h
        self.n_in, self.hidden, self.n_out = n_in, hidden, n_out
        c = ctypes.c_int()
        _check(lib().ift_mlp_num_params(h, ctypes.byref(c)), "ift_mlp_num_params")
        self.n_params = c.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.ift_mlp_destroy(h)
            self.handle = None

    def set_params(self, params, stream=None):
        import torch
        _check(lib().ift_mlp_set_params(self.handle, _ptr(params, self.n_params, torch.float32), _stream(stream)),
               "ift_mlp_set_params")

    def get_params(self, params, stream=None):
        import torch
        _check(lib().ift_mlp_get_params(self.handle, _ptr(params, self.n_params, torch.float32), _stream(stream)),
               "ift_mlp_get_params")

    def set_normalization(self, x_mean, x_scale, y_mean, y_scale):
        a = [np.ascontiguousarray(v, dtype=np.float64) for v in (x_mean, x_scale, y_mean, y_scale)]
        _check(lib().ift_mlp_set_normalization(self.handle, *[v.ctypes.data_as(_D) for v in a]),
               "ift_mlp_set_normalization")

    def loss_grad(self, X, T, grad=None, stream=None):
        import torch
        N = int(X.shape[0])
        loss = ctypes.c_double()
        _check(lib().ift_mlp_loss_grad(self.handle, _ptr(X, N * self.n_in, torch.float32),
                                       _ptr(T, N * self.n_out, torch.float32), N,
                                       _ptr(grad, self.n_params, torch.float32), ctypes.byref(loss),
                                       _stream(stream)), "ift_mlp_loss_grad")
        return loss.value

    def train(self, mu, z, steps, lr=1e-3, stream=None):
        import torch
        N = int(mu.shape[0])
        hist = np.zeros(max(steps, 1))
        _check(lib().ift_mlp_train(self.handle, _ptr(mu, N * self.n_in, torch.float64),
                                   _ptr(z, N * self.n_out, torch.float64), N, int(steps), float(lr),
                                   hist.ctypes.data_as(_D), _stream(stream)), "ift_mlp_train")
        return hist[:steps]

    def predict(self, mu, z, bf16=True, stream=None):
        import torch
        N = int(mu.shape[0])
        _check(lib().ift_mlp_predict(self.handle, _ptr(mu, N * self.n_in, torch.float64), N,
                                     _ptr(z, N * self.n_out, torch.float64), int(bool(bf16)), _stream(stream)),
               "ift_mlp_predict")


def profile_enable(on: bool = True):
    _check(lib().ift_profile_enable(int(bool(on))), "ift_profile_enable")


def profile_reset():
    _check(lib().ift_profile_reset(), "ift_profile_reset")


def profile_read(which: str):
    """(launch count, total milliseconds) of one kernel class since the last reset."""
    c, ms = ctypes.c_int(), ctypes.c_double()
    _check(lib().ift_profile_read(PROF[which], ctypes.byref(c), ctypes.byref(ms)), "ift_profile_read")
    return c.value, ms.value


# names matching the C ABI
def hdm_assemble(prob: Problem, *a, **k):
    return prob.hdm_assemble(*a, **k)


def eq_assemble_residual(rom: ROM, *a, **k):
    return rom.eq_assemble_residual(*a, **k)


def rom_gauss_newton_solve_batched(batch: Batch, *a, **k):
    return batch.solve(*a, **k)


def eq_assemble_jacobian_batched(batch: Batch, *a, **k):
    return batch.eq_assemble_jacobian(*a, **k)


def eq_assemble_jacobian(rom: ROM, *a, **k):
    return rom.eq_assemble_jacobian(*a, **k)


def rom_gauss_newton_step(rom: ROM, *a, **k):
    return rom.gauss_newton_step(*a, **k)
