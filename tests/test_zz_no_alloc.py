"""eq_assemble_jacobian_noalloc (static device scratch, no allocation)
against eq_assemble_jacobian through the C ABI: the same kernels, so the
objective, gradient, Gauss-Newton matrix and invalid count agree to the last
bit.  Two calls in a row on the same device, the second on a ROM with a
smaller EQ set (the scratch keeps the first call's contents), and a ROM
whose workspace exceeds the scratch is refused."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _both(rom, mu, w, tau, dev):
    import torch
    f64 = torch.float64
    out = []
    for noalloc in (False, True):
        J = torch.full((1,), np.nan, dtype=f64, device=dev)
        g = torch.full((rom.D,), np.nan, dtype=f64, device=dev)
        H = torch.full((rom.D * rom.D,), np.nan, dtype=f64, device=dev)
        nb = torch.full((1,), -1, dtype=torch.int32, device=dev)
        wt, tt = torch.tensor(w, device=dev), torch.tensor(tau, device=dev)
        if noalloc:
            rom.eq_assemble_jacobian_noalloc(mu, wt, tt, J, g, H, nb)
        else:
            rom.eq_assemble_jacobian(mu, wt, tt, J, g, H, None, nb)
        torch.cuda.synchronize()
        out.append((J.cpu().numpy(), g.cpu().numpy(), H.cpu().numpy(), nb.cpu().numpy()))
    return out


def test_noalloc_matches_allocating_entry_point():
    import torch
    from paper_2305_15661_amd import ift
    dev = torch.device("cuda:0")
    base = synth.euler_p2(nx=16, ny=8, n=20, m=10, n_s=64)
    prob = ift.Problem.from_workload(base)
    Phi = torch.tensor(base.Phi, device=dev)
    Psi = torch.tensor(base.Psi, device=dev)
    rng = np.random.default_rng(77)
    # a larger EQ set first, then a smaller one
    for ns in (200, 37):
        el = np.sort(rng.choice(base.mesh.n_elem, ns, replace=False))
        rho = rng.lognormal(0.0, 0.5, size=ns)
        rom = ift.ROM(prob, Phi, Psi, el, rho)
        assert 0 < rom.noalloc_scratch_bytes() <= ift.NOALLOC_SCRATCH_BYTES
        for k in range(2):
            _say(f"no-alloc assembly: n_s {ns}, point {k}")
            (J0, g0, H0, n0), (J1, g1, H1, n1) = _both(rom, base.mus[k], base.w_eval[k], base.tau_eval[k], dev)
            assert np.isfinite(J0).all() and np.isfinite(g0).all() and np.isfinite(H0).all()
            assert np.array_equal(J1, J0) and np.array_equal(g1, g0) and np.array_equal(H1, H0)
            assert np.array_equal(n1, n0)


def test_noalloc_refuses_oversized_workspace():
    import torch
    from paper_2305_15661_amd import ift
    dev = torch.device("cuda:0")
    base = synth.euler_p2(nx=64, ny=48, n=10, m=5, n_s=64)   # 6144 elements
    prob = ift.Problem.from_workload(base)
    el = np.arange(base.mesh.n_elem)
    rom = ift.ROM(prob, torch.tensor(base.Phi, device=dev), torch.tensor(base.Psi, device=dev), el,
                  np.ones(el.size))
    assert rom.noalloc_scratch_bytes() > ift.NOALLOC_SCRATCH_BYTES
    J = torch.zeros(1, dtype=torch.float64, device=dev)
    g = torch.zeros(rom.D, dtype=torch.float64, device=dev)
    H = torch.zeros(rom.D * rom.D, dtype=torch.float64, device=dev)
    _say("no-alloc assembly: oversized ROM")
    with pytest.raises(ift.IftError) as ei:
        rom.eq_assemble_jacobian_noalloc(base.mus[0], torch.tensor(base.w_eval[0], device=dev),
                                         torch.tensor(base.tau_eval[0], device=dev), J, g, H)
    assert ei.value.status == ift.IFT_ESCRATCH
