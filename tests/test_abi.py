"""The C-ABI library loads, exports every symbol of include/ift.h, and
rejects bad arguments on the host before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2305_15661_amd import ift
    if not os.path.exists(ift.LIB_PATH):
        pytest.fail("libift.so not built: run paper_2305_15661_amd/build.py")
    return ift, ift.lib()


def test_every_declared_symbol_is_exported():
    ift, L = _lib()
    hdr = open(os.path.join(ROOT, "include", "ift.h")).read()
    names = set(re.findall(r"^(?:ift_status|void|size_t)\s+(\w+)\s*\(", hdr, flags=re.M))
    assert names == set(ift.EXPORTS), names ^ set(ift.EXPORTS)
    for n in names:
        assert hasattr(L, n)


def _desc(ift, wl, **over):
    X = np.ascontiguousarray(wl.mesh.X.reshape(-1))
    gn = np.ascontiguousarray(wl.mesh.elem_gnodes, dtype=np.int32)
    nb = np.ascontiguousarray(wl.mesh.elem_nbr, dtype=np.int32)
    kw = dict(pde=ift.PDE[wl.pde], p=wl.p, n_elem=gn.shape[0], n_gnode=X.size // 2, gamma=1.4, kappa=0.1,
              eps_g=1e-8, bc_mu_scale=0.5, all_farfield=0, src_amp=0.0, bc_spacetime=0)
    kw.update(over)
    d = ift.ProblemDesc(kw["pde"], kw["p"], kw["n_elem"], kw["n_gnode"], X.ctypes.data_as(ift._D),
                        gn.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), nb.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                        kw["gamma"], kw["kappa"], kw["eps_g"], kw["bc_mu_scale"], kw["all_farfield"],
                        kw["src_amp"], kw["bc_spacetime"])
    return d, (X, gn, nb)


@pytest.mark.parametrize("over", [dict(p=3), dict(pde=7), dict(n_elem=0), dict(eps_g=0.0), dict(kappa=-1.0),
                                  dict(gamma=1.0, pde=1), dict(src_amp=float("nan")), dict(bc_spacetime=2),
                                  dict(pde=1, src_amp=0.02), dict(pde=1, bc_spacetime=1)])
def test_bad_descriptor_rejected(over):
    ift, L = _lib()
    wl = synth.tiny_burgers()
    d, keep = _desc(ift, wl, **over)
    h = ctypes.c_void_p()
    assert L.ift_problem_create(ctypes.byref(d), ctypes.byref(h)) == ift.IFT_EINVAL
    assert not h.value


def test_bad_mesh_rejected():
    ift, L = _lib()
    wl = synth.tiny_burgers()
    for mut in ("nonmutual", "range", "tag", "orientation"):
        d, (X, gn, nb) = _desc(ift, wl)
        if mut == "nonmutual":
            nb[0, 2] = 5
        elif mut == "range":
            gn[3, 1] = 10 ** 6
        elif mut == "tag":
            nb[0, 0] = -9
        else:
            gn[1, [0, 1]] = gn[1, [1, 0]]
        h = ctypes.c_void_p()
        assert L.ift_problem_create(ctypes.byref(d), ctypes.byref(h)) == ift.IFT_EINVAL, mut


def test_null_handles_rejected():
    ift, L = _lib()
    mu = (ctypes.c_double * 2)(0.3, 0.0)
    assert L.hdm_assemble(None, mu, None, None, None, None, None, None, None, None, None, None) == ift.IFT_EINVAL
    assert L.eq_assemble_residual(None, mu, None, None, None, None, None, None, None) == ift.IFT_EINVAL
    assert L.eq_assemble_jacobian(None, mu, None, None, None, None, None, None, None, None) == ift.IFT_EINVAL
    assert L.rom_gauss_newton_step(None, mu, None, None, None, None, None) == ift.IFT_EINVAL
    assert L.ift_rom_get_gathers(None, None, None, None, None, None) == ift.IFT_EINVAL
    assert L.ift_problem_neighbour_map(None, None) == ift.IFT_EINVAL
    L.ift_problem_destroy(None)
    L.ift_rom_destroy(None)


def test_batch_arguments_rejected():
    ift, L = _lib()
    h = ctypes.c_void_p()
    arr = (ctypes.c_void_p * 2)(None, None)
    assert L.ift_batch_create(0, arr, ctypes.byref(h)) == ift.IFT_EINVAL
    assert L.ift_batch_create(2, arr, ctypes.byref(h)) == ift.IFT_EINVAL
    assert L.ift_batch_create(1, None, ctypes.byref(h)) == ift.IFT_EINVAL
    assert not h.value
    assert L.ift_batch_layout(None, None, None) == ift.IFT_EINVAL
    assert L.ift_batch_autotune(None, None, None, None, None) == ift.IFT_EINVAL
    assert L.eq_assemble_jacobian_batched(None, None, None, None, None, None, None, None) == ift.IFT_EINVAL
    prm = ift.GNParams(0.0, 1e-4, 30, 1e-8)
    assert L.rom_gauss_newton_solve_batched(None, None, None, ctypes.byref(prm), 10, None, 0, None) == ift.IFT_EINVAL
    L.ift_batch_destroy(None)


def test_mlp_arguments_rejected():
    ift, L = _lib()
    h = ctypes.c_void_p()
    for args in ((0, 16, 4), (2, 0, 4), (2, 16, 0), (9, 16, 4), (2, 300, 4), (2, 16, 65)):
        assert L.ift_mlp_create(*args, 1, ctypes.byref(h)) == ift.IFT_EINVAL
        assert not h.value
    assert L.ift_mlp_train(None, None, None, 1, 1, 1e-3, None, None) == ift.IFT_EINVAL
    assert L.ift_mlp_predict(None, None, 1, None, 0, None) == ift.IFT_EINVAL
    L.ift_mlp_destroy(None)


def test_residual_norm_arguments_rejected():
    ift, L = _lib()
    assert L.hdm_residual_norm_batched(None, 1, None, None, 1, None, None, 0, None, None, None, None) == ift.IFT_EINVAL


def test_greedy_select_ranks_invalid_candidates_first():
    from paper_2305_15661_amd import ift
    # host-side argmax of eq. (greedy0): an invalid lifted state (+inf or
    # NaN norm) is the candidate most in need of a full-order solve
    assert ift.greedy_select(np.array([0.1, 3.0, 2.0])) == 1
    assert ift.greedy_select(np.array([0.1, 3.0, np.inf, np.nan])) == 2
    assert ift.greedy_select(np.array([0.1, np.nan, 3.0])) == 1


def test_bench_refuses_several_gpus():
    # one GPU per process: the benchmark says so instead of running
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
