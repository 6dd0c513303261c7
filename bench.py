"""Benchmark of the EQ-hyperreduced assembly on one MI355X.

Workload: P2 compressible Euler on a 128x64-cell mesh of [0,2]x[0,1]
(16384 elements), reduced bases n = 20 (state) and m = 10 (mapping), 819
EQ-sampled elements with lognormal(0, 0.5) weights, FP64.  Inputs are
seeded synthetic data (see synth/); they stay resident in HBM.

A step is one batched eq_assemble_jacobian call over the 16 seeded
evaluation points (mu, w, tau) of the workload: per sampled element and
point, the lift, mapped geometry, DG volume and face terms with exact point
Jacobians, the projection onto [Phi_e; Phi_e'] and Psi_e, and the
rho-weighted Gram reduction to the Gauss-Newton matrix and gradient.
value = sampled element-evals per second (16 x n_s per step).  The line
also carries:
  solves_per_s   Gauss-Newton solves to |S~|,|T~| <= 1e-8 from the 16
                 seeded evaluation points (each a rom_gauss_newton_step
                 loop including line searches);
  hdm_assemble   the full-order element loop over all 16384 elements with
                 all Jacobian blocks (evals/s);
  roofline       for the kernel with the largest share of the step time,
                 timed with HIP events bracketing its launches on the
                 caller's stream;
  cpu_baseline   the CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "EQ residual+Jacobian element-evals/s; ROM Gauss-Newton solves/s to ||r||<=1e-8"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6

# Algorithmic work per sampled element-eval at nue = 24, nun = 36, nxe = 12,
# n = 20, m = 10 (FP64), split over the kernels of the Jacobian path:
#  points (lift, geometry, DG volume/face terms, distortion with exact point
#          Jacobians): reads the gathered EQ operands Phi_e 24x20,
#          Phi_e' 36x20, Psi_e 12x10, X_e 12 and rho/ids (10,680 B);
#  eq_jac (projection and weighting, fused with the Gram reduction): the
#          contraction A^U = J^U Phi_e + J^U' Phi_e' (2*24*60*20 = 57,600),
#          A^x = J^x Psi_e (2*24*12*10 = 5,760), H += A^T A (2*25*30*30 =
#          45,000 with the distortion row; 43,200 without it) and g
#          (2*25*30 = 1,500): 108,000 counted as in the path table;
#  gram   (sum of the per-block partials): bytes of the partials read.
KBYTES = {"points": 8 * (24 * 20 + 36 * 20 + 12 * 10 + 12) + 24,
          "eq_jac": 8 * (24 * 20 + 36 * 20 + 12 * 10),
          "gram": 8 * 25 * 31}
KFLOPS = {"points": None,
          "eq_jac": 57600 + 5760 + 43200 + 1440,
          "gram": None}
KNAMES = {"points": "k_phys_points + k_points_eq2<Euler P2, fp64>", "eq_jac": "k_eq_fused_pts2<Euler P2, fp64, 2, 11>",
          "gram": "k_fused_final"}
# HBM traffic per launch of each kernel from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch) on this workload, scaled by what the same
# counters read for a plain copy kernel of known size (a 512 MiB copy reads
# back as 256 MiB fetched and 512 MiB written:
# profiles/hbm_counter_calibration_copy_512mib.md).  These are the counters
# of profiles/eq_jacobian_euler_p2_819x16.md, taken on the kernels as they
# now stand; an entry must become None when its kernel changes.
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
TRAFFIC_KIB = {"points": (4511.6, 80570.2), "eq_jac": (48737.4, 6176.0), "gram": (4897.5, 290.7)}
TRAFFIC_SOURCE = "profiles/eq_jacobian_euler_p2_819x16.md"
# the full-order kernel (profiles/hdm_assemble_euler_p2_16384.md)
HDM_TRAFFIC_KIB = (9551.2, 226304.0)
# Full-order loop with Jacobians: reads U_e, the neighbour traces, x_e, X_e
# and connectivity; writes R_e, N_e, dR/dU_e, dR/dU_e', dR/dx_e, dN/dx_e.
HDM_BYTES_PER_ELEM = 8 * (24 + 36 + 12 + 12) + 4 * (6 + 3 + 36) + 8 * (24 + 1 + 24 * 24 + 24 * 36 + 24 * 12 + 12)


PEAK_BF16_TFLOPS = 2500.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def batch_work(bw, n_inst, mixed=False):
    """Algorithmic bytes and flops of one batched Jacobian phase, summed over
    the instances (n_s, n, m of each; nue = 24, nun = 36, nxe = 12):
    bytes: the gathered operands Phi_e, Phi_e', Psi_e, X_e and rho/ids (FP64;
    with mixed precision Phi in BF16 and Psi, X in FP32); projection flops
    A^U 2*24*60*n + A^x 2*24*12*m; Gram flops H 2*24*D^2 + g 2*24*D."""
    by = proj = gram = 0.0
    for i in range(n_inst):
        ns = bw.inst_elem[i].size
        n, m = bw.pool_nm[bw.inst_pool[i]]
        D = n + m
        bphi, bpsi = (2, 4) if mixed else (8, 8)
        by += ns * (bphi * 60 * n + bpsi * (12 * m + 12) + 24)
        proj += ns * (2 * 24 * 60 * n + 2 * 24 * 12 * m)
        gram += ns * (2 * 24 * D * D + 2 * 24 * D)
    return by, proj, gram


def batch_roofline(b, mu, z, by, proj, gram, reps, mixed=False):
    """Per-kernel HIP-event times of the batched Jacobian phase (points,
    projection + Gram, final sums) and their roofline fractions."""
    import torch
    from paper_2305_15661_amd import ift
    dev = z.device
    J = torch.zeros(b.n_inst, dtype=torch.float64, device=dev)
    g = torch.zeros(b.nz, dtype=torch.float64, device=dev)
    H = torch.zeros(b.nh, dtype=torch.float64, device=dev)
    b.eq_assemble_jacobian(mu, z, J, g, H)
    torch.cuda.synchronize()
    ift.profile_enable(True)
    ift.profile_reset()
    for _ in range(reps):
        b.eq_assemble_jacobian(mu, z, J, g, H)
    torch.cuda.synchronize()
    ift.profile_enable(False)
    t = {k: ift.profile_read(k)[1] * 1e-3 / reps for k in ("points", "eq_jac", "gram")}
    pts_gbs = by / t["points"] / 1e9
    proj_peak = PEAK_BF16_TFLOPS if mixed else PEAK_FP64_TFLOPS
    out = {"kernels_us": {k: v * 1e6 for k, v in t.items()},
           "phase_us": sum(t.values()) * 1e6,
           "algorithmic_bytes": by, "projection_flops": proj, "gram_flops": gram,
           "points": {"bound": "hbm", "achieved": pts_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                      "frac": pts_gbs / PEAK_HBM_GBS},
           "projection": {"bound": "mfma", "unit": "TFLOP/s",
                          "projection_achieved": proj / t["eq_jac"] / 1e12, "projection_peak": proj_peak,
                          "projection_frac": proj / t["eq_jac"] / 1e12 / proj_peak,
                          "gram_achieved": gram / t["eq_jac"] / 1e12, "gram_peak": PEAK_FP64_TFLOPS,
                          "gram_frac": gram / t["eq_jac"] / 1e12 / PEAK_FP64_TFLOPS},
           "phase_hbm_frac": by / sum(t.values()) / 1e9 / PEAK_HBM_GBS}
    if not mixed:
        tf = (proj + gram) / t["eq_jac"] / 1e12
        out["projection"].update({"achieved": tf, "peak": PEAK_FP64_TFLOPS, "frac": tf / PEAK_FP64_TFLOPS})
    return out


def host_info():
    """The host the oracle runs on: core count, CPU model, BLAS and versions."""
    import platform

    import scipy
    from threadpoolctl import threadpool_info
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_count": os.cpu_count(), "cpus_usable": len(os.sched_getaffinity(0)), "cpu_model": model,
            "machine": platform.machine(), "numpy": np.__version__, "scipy": scipy.__version__,
            "blas": [{"api": d.get("internal_api"), "threads": d.get("num_threads"), "version": d.get("version")}
                     for d in threadpool_info()]}


def _timed(fn, budget_s: float, min_runs: int = 1, max_runs: int = 5):
    """Median wall time of fn() over up to max_runs runs after one warm-up,
    stopping once budget_s is spent (at least min_runs runs)."""
    fn()
    ts = []
    t_all = time.perf_counter()
    while len(ts) < max_runs and (len(ts) < min_runs or time.perf_counter() - t_all < budget_s):
        t = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts)), len(ts)


def cpu_baseline(wl, budget_s: float, full: bool = False):
    """The oracle (plain FP64 NumPy/SciPy, vectorised over elements, not tuned)
    on the host cores, with one BLAS thread and with the host's default
    thread count: the C1 EQ Jacobian assembly (the headline unit), a sample
    of the full-order assembly, and the C0 Gauss-Newton solve; with full=True
    also a C1 solve and batched-workload instances solved one by one."""
    from threadpoolctl import threadpool_info, threadpool_limits

    import synth
    from oracle import eq as oeq
    from oracle import gn as ogn
    from oracle import residual as ors
    prob = ors.Problem(wl)
    orom = oeq.ROM(prob, wl.Phi, wl.Psi, wl.eq_elem, wl.eq_rho)
    wl0 = synth.tiny_burgers()
    orom0 = oeq.ROM(ors.Problem(wl0), wl0.Phi, wl0.Psi, wl0.eq_elem, wl0.eq_rho)
    w00, t00 = oeq.plain_start(wl0, wl0.mus[0])
    U = wl.Phi @ wl.w_eval[0]
    x = wl.X + wl.Psi @ wl.tau_eval[0]
    chunk = np.arange(1024)
    Ue, Une, xe = prob.gather_state(chunk, U, x)
    runs = {}
    for label, limit in (("1_thread", 1), ("default_threads", None)):
        with threadpool_limits(limit):
            threads = max([d.get("num_threads") or 1 for d in threadpool_info()] or [1])
            k = [0]

            def jac():
                j = k[0] % wl.mus.shape[0]
                k[0] += 1
                orom.jacobian(wl.mus[j], wl.w_eval[j], wl.tau_eval[j])
            t_jac, n_jac = _timed(jac, budget_s / 2, min_runs=3, max_runs=50)
            t_hdm, n_hdm = _timed(lambda: prob.evaluate(chunk, Ue, Une, xe, wl.mus[0], True), budget_s / 8, 1, 3)
            t_c0, n_c0 = _timed(lambda: ogn.lm_solve(orom0, wl0.mus[0], w00, t00, 0.0, 1e-8, 20), budget_s / 8, 5, 5)
            r = {"threads": threads,
                 "eq_jacobian_c1": {"element_evals_per_s": wl.n_s / t_jac, "ms_per_call": t_jac * 1e3,
                                    "runs": n_jac, "statistic": "median"},
                 "hdm_assemble_c1_sample": {"elements": int(chunk.size), "element_evals_per_s": chunk.size / t_hdm,
                                            "seconds_per_call_full_mesh_est": t_hdm * wl.mesh.n_elem / chunk.size,
                                            "runs": n_hdm},
                 "gn_solve_c0": {"ms_per_solve": t_c0 * 1e3, "solves_per_s": 1.0 / t_c0, "runs": n_c0,
                                 "iterations": 20}}
            if full:
                t_c1, _ = _timed(lambda: ogn.lm_solve(orom, wl.mus[0], wl.w_eval[0], wl.tau_eval[0], 0.0, 1e-8, 60),
                                 0.0, 1, 1)
                r["gn_solve_c1"] = {"seconds_per_solve": t_c1, "solves_per_s": 1.0 / t_c1, "runs": 1}
                if limit == 1:
                    r["batched_loop"] = cpu_batched_loop(n=4)
            runs[label] = r
            log(f"cpu ({label}, {threads} threads): eq jacobian {wl.n_s / t_jac:.0f} evals/s, "
                f"hdm sample {chunk.size / t_hdm:.0f} evals/s, C0 solve {t_c0 * 1e3:.0f} ms")
    best = max(runs.values(), key=lambda r: r["eq_jacobian_c1"]["element_evals_per_s"])
    return {"value": best["eq_jacobian_c1"]["element_evals_per_s"], "unit": "element-evals/s",
            "cores": best["threads"], "kind": "oracle",
            "sample": (f"oracle eq_assemble_jacobian on the same 16384-element Euler P2 workload (819 EQ elements, "
                       f"median of {best['eq_jacobian_c1']['runs']} calls over the 16 evaluation points) with "
                       f"{best['threads']} BLAS thread(s); also 1-thread and default-thread runs of a 1024-element "
                       f"full-order sample and of the C0 Gauss-Newton solve"),
            "host": host_info(), "runs": runs}


def cpu_batched_loop(n: int):
    """The oracle's Levenberg-Marquardt solves of the first n batched-workload
    instances, one after the other (the count is stated, not extrapolated)."""
    import dataclasses

    import synth
    from oracle import eq as oeq
    from oracle import gn as ogn
    from oracle import residual as ors
    bw = synth.euler_batch(n_inst=max(n, 1))
    prob = ors.Problem(bw.base)
    t = time.perf_counter()
    conv, its = 0, []
    for i in range(n):
        P, S = bw.pool[bw.inst_pool[i]]
        wl = synth.with_eq(bw.base, bw.inst_elem[i], bw.inst_rho[i])
        orom = oeq.ROM(prob, P, S, bw.inst_elem[i], bw.inst_rho[i])
        w0, t0 = oeq.plain_start(dataclasses.replace(wl, Phi=P, Psi=S), bw.mus[i])
        _, _, info = ogn.lm_solve(orom, bw.mus[i], w0, t0, BATCH_LAMBDA, 1e-8, BATCH_MAX_IT)
        conv += info["status"] == "converged"
        its.append(info["iterations"])
    dt = time.perf_counter() - t
    return {"instances": n, "converged": conv, "seconds": dt, "solves_per_s": conv / dt,
            "mean_gn_iterations": float(np.mean(its))}


BATCH_LAMBDA = 1e-10   # Levenberg-Marquardt weight on the mapping block
BATCH_MAX_IT = 50


def batched_leg(n_inst: int, n_loop: int, dev):
    """Batched solves of many instances (pool of 6 bases with n in
    {10, 20, 30}, m in {5, 10}; EQ sets of U{200..2000} elements plus the
    inflow elements; mu = (Mach, angle) from a scrambled Sobol sequence on
    [2, 3] x [-5, 5] degrees), all from the plain start, versus a loop of
    rom_gauss_newton_step over the first n_loop instances."""
    import torch
    import synth
    from paper_2305_15661_amd import ift
    t0 = time.perf_counter()
    bw = synth.euler_batch(n_inst=n_inst)
    prob = ift.Problem.from_workload(bw.base)
    pool = [(torch.tensor(np.ascontiguousarray(P), device=dev), torch.tensor(np.ascontiguousarray(S), device=dev))
            for P, S in bw.pool]
    roms = [ift.ROM(prob, *pool[bw.inst_pool[i]], bw.inst_elem[i], bw.inst_rho[i]) for i in range(n_inst)]
    b = ift.Batch(roms)
    torch.cuda.synchronize()
    log(f"batched leg: setup {time.perf_counter() - t0:.1f} s")
    ns = int(sum(e.size for e in bw.inst_elem))
    mu = torch.tensor(bw.mus, dtype=torch.float64, device=dev)
    z0 = torch.zeros(b.nz, dtype=torch.float64, device=dev)
    b.plain_start(mu, z0)
    E = b.autotune(mu, z0)
    # Jacobian assembly over the whole batch
    J = torch.zeros(n_inst, dtype=torch.float64, device=dev)
    g = torch.zeros(b.nz, dtype=torch.float64, device=dev)
    H = torch.zeros(b.nh, dtype=torch.float64, device=dev)
    for _ in range(2):
        b.eq_assemble_jacobian(mu, z0, J, g, H)
    torch.cuda.synchronize()
    reps = 5
    t = time.perf_counter()
    for _ in range(reps):
        b.eq_assemble_jacobian(mu, z0, J, g, H)
    torch.cuda.synchronize()
    t_jac = (time.perf_counter() - t) / reps
    by64, proj64, gram64 = batch_work(bw, n_inst)
    roof2 = batch_roofline(b, mu, z0, by64, proj64, gram64, reps)
    log(f"batched jacobian (FP64): points {roof2['kernels_us']['points']:.0f} us, projection + Gram "
        f"{roof2['kernels_us']['eq_jac']:.0f} us ({roof2['projection']['frac']:.3f} of FP64), final "
        f"{roof2['kernels_us']['gram']:.0f} us; phase {roof2['phase_hbm_frac']:.3f} of HBM")
    # solves (graph replay); the first call captures the graph
    info = b.info_buffer(dev)
    z = z0.clone()
    b.solve(mu, z, info, lam=BATCH_LAMBDA, max_it=BATCH_MAX_IT)
    torch.cuda.synchronize()
    z = z0.clone()
    torch.cuda.synchronize()
    t = time.perf_counter()
    b.solve(mu, z, info, lam=BATCH_LAMBDA, max_it=BATCH_MAX_IT)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t
    o = ift.Batch.info_array(info)
    z64 = b.unpack(z)
    conv = int(o["converged"].sum())
    st, cnt = np.unique(o["status"], return_counts=True)
    # mixed precision on the same instances: FP32 physics, BF16 projection,
    # FP64 Gram and solves, FP64 refinement rounds
    romsm = [ift.ROM(prob, *pool[bw.inst_pool[i]], bw.inst_elem[i], bw.inst_rho[i], "mixed") for i in range(n_inst)]
    bm = ift.Batch(romsm)
    bm.autotune(mu, z0)
    byb, projb, gramb = batch_work(bw, n_inst, mixed=True)
    roof3 = batch_roofline(bm, mu, z0, byb, projb, gramb, reps, mixed=True)
    log(f"batched jacobian (mixed): points {roof3['kernels_us']['points']:.0f} us, projection + Gram "
        f"{roof3['kernels_us']['eq_jac']:.0f} us ({roof3['projection']['projection_frac']:.4f} of BF16, "
        f"Gram {roof3['projection']['gram_frac']:.3f} of FP64); phase {roof3['phase_hbm_frac']:.3f} of HBM")
    infom = bm.info_buffer(dev)
    zm = z0.clone()
    bm.solve(mu, zm, infom, lam=BATCH_LAMBDA, max_it=BATCH_MAX_IT)
    torch.cuda.synchronize()
    zm = z0.clone()
    torch.cuda.synchronize()
    t = time.perf_counter()
    bm.solve(mu, zm, infom, lam=BATCH_LAMBDA, max_it=BATCH_MAX_IT)
    torch.cuda.synchronize()
    t_mixed = time.perf_counter() - t
    om = ift.Batch.info_array(infom)
    convm = int(om["converged"].sum())
    zmu = bm.unpack(zm)
    del bm, romsm
    # accuracy: both solves stop at |S~|, |T~| <= 1e-8, which fixes the
    # iterate only to about |H^-1| * 1e-8; each is compared with a tight FP64
    # solve (tol 1e-11) of the same instance, in z and in w (Phi has
    # orthonormal columns, so |w - w*| / |w*| = |Phi (w - w*)| / |Phi w*|)
    zr = z0.clone()
    b.solve(mu, zr, info, lam=BATCH_LAMBDA, max_it=4 * BATCH_MAX_IT, tol=1e-11)
    torch.cuda.synchronize()
    oref = ift.Batch.info_array(info)
    zref = b.unpack(zr)

    def err_stats(zs, conv):
        ez, ew = [], []
        for i in range(n_inst):
            if conv[i] and oref["converged"][i]:
                n_i = bw.pool_nm[bw.inst_pool[i]][0]
                ez.append(np.linalg.norm(zs[i] - zref[i]) / np.linalg.norm(zref[i]))
                ew.append(np.linalg.norm(zs[i][:n_i] - zref[i][:n_i]) / np.linalg.norm(zref[i][:n_i]))
        ez, ew = np.array(ez), np.array(ew)
        if not ez.size:
            return None
        return {"instances": int(ez.size), "z_median": float(np.median(ez)), "z_p90": float(np.quantile(ez, 0.9)),
                "z_max": float(ez.max()), "z_fraction_le_1e-6": float(np.mean(ez <= 1e-6)),
                "w_median": float(np.median(ew)), "w_max": float(ew.max()),
                "w_fraction_le_1e-6": float(np.mean(ew <= 1e-6))}

    acc = {"reference": f"FP64 batch to tol 1e-11 ({int(oref['converged'].sum())} of {n_inst} converged within "
                        f"{4 * BATCH_MAX_IT} iterations)",
           "fp64_tol_1e-8": err_stats(z64, o["converged"]), "mixed_tol_1e-8": err_stats(zmu, om["converged"])}
    mixed = {"solves_per_s": convm / t_mixed, "converged": convm, "seconds": t_mixed,
             "mean_gn_iterations": float(om["iterations"].mean()),
             "mean_mixed_precision_iterations": float(om["mixed_iterations"].mean()),
             "speedup_vs_fp64_batch": (convm / t_mixed) / (conv / t_solve) if conv else None,
             "error_vs_tight_fp64": acc, "roofline_jacobian_phase": roof3}
    am = acc["mixed_tol_1e-8"] or {}
    af = acc["fp64_tol_1e-8"] or {}
    log(f"mixed: {convm} converged in {t_mixed:.3f} s ({convm / t_mixed:.1f} solves/s), "
        f"{mixed['mean_mixed_precision_iterations']:.1f} of {mixed['mean_gn_iterations']:.1f} steps mixed; "
        f"error vs tight FP64: mixed z median {am.get('z_median')}, w median {am.get('w_median')}; "
        f"fp64 z median {af.get('z_median')}, w median {af.get('w_median')}")
    log(f"batched: {n_inst} instances, {conv} converged in {t_solve:.3f} s ({conv / t_solve:.1f} solves/s), "
        f"jacobian {t_jac * 1e3:.2f} ms ({ns / t_jac:.3e} evals/s), E={E}")
    # greedy indicator, eq. (greedy0), at every FP64 solution: full-order
    # residual norms over all elements, grouped by the pool basis
    groups = []
    for pidx in range(len(pool)):
        ids = [i for i in range(n_inst) if bw.inst_pool[i] == pidx]
        if not ids:
            continue
        n_p, m_p = bw.pool_nm[pidx]
        wz = torch.tensor(np.stack([z64[i][:n_p] for i in ids]), device=dev)
        tz = torch.tensor(np.stack([z64[i][n_p:] for i in ids]), device=dev)
        mz = torch.tensor(bw.mus[ids], dtype=torch.float64, device=dev)
        groups.append((ids, pidx, mz, wz, tz, torch.zeros(len(ids), dtype=torch.float64, device=dev)))
    for _ in range(2):
        for ids, pidx, mz, wz, tz, nz in groups:
            prob.hdm_residual_norms(mz, pool[pidx][0], wz, pool[pidx][1], tz, nz)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for ids, pidx, mz, wz, tz, nz in groups:
        prob.hdm_residual_norms(mz, pool[pidx][0], wz, pool[pidx][1], tz, nz)
    torch.cuda.synchronize()
    t_greedy = time.perf_counter() - t
    norms = np.zeros(n_inst)
    for ids, pidx, mz, wz, tz, nz in groups:
        norms[ids] = nz.cpu().numpy()
    best = ift.greedy_select(norms)
    n_elem = bw.base.mesh.n_elem
    greedy = {"candidates": n_inst, "elements": n_elem, "seconds": t_greedy,
              "element_evals_per_s": n_inst * n_elem / t_greedy, "argmax": best,
              "mu_argmax": [float(v) for v in bw.mus[best]], "norm_max": float(norms[best]),
              "invalid_candidates": int(np.count_nonzero(~np.isfinite(norms)))}
    log(f"greedy indicator: {n_inst} candidates x {n_elem} elements in {t_greedy * 1e3:.1f} ms "
        f"({greedy['element_evals_per_s']:.3e} element-evals/s); next parameter {greedy['mu_argmax']}")
    # the same FP64 batch with the paper's initialisation (steps in w with
    # tau held until |S~| <= tol, then full steps)
    zp = z0.clone()
    b.solve(mu, zp, info, lam=BATCH_LAMBDA, max_it=BATCH_MAX_IT, presolve=True)
    torch.cuda.synchronize()
    zp = z0.clone()
    torch.cuda.synchronize()
    t = time.perf_counter()
    b.solve(mu, zp, info, lam=BATCH_LAMBDA, max_it=BATCH_MAX_IT, presolve=True)
    torch.cuda.synchronize()
    t_pre = time.perf_counter() - t
    op = ift.Batch.info_array(info)
    convp = int(op["converged"].sum())
    presolve = {"solves_per_s": convp / t_pre, "converged": convp, "seconds": t_pre,
                "mean_gn_iterations": float(op["iterations"].mean()),
                "mean_w_only_iterations": float(op["presolve_iterations"].mean())}
    log(f"batched with w-only initialisation: {convp} converged in {t_pre:.3f} s ({convp / t_pre:.1f} solves/s), "
        f"{presolve['mean_w_only_iterations']:.1f} of {presolve['mean_gn_iterations']:.1f} steps in w")
    # per-instance loop of the same FP64 path on the first n_loop instances
    t = time.perf_counter()
    lconv, lits = 0, []
    for i in range(min(n_loop, n_inst)):
        r = roms[i]
        w = torch.zeros(r.n, dtype=torch.float64, device=dev)
        tau = torch.zeros(r.m, dtype=torch.float64, device=dev)
        r.plain_start(bw.mus[i], w, tau)
        steps = 0
        while True:
            last = steps == BATCH_MAX_IT
            wc, tc = (w.clone(), tau.clone()) if last else (w, tau)
            st_, inf_ = r.gauss_newton_step(bw.mus[i], wc, tc, lam=BATCH_LAMBDA)
            if inf_["converged"] or st_ != 0 or last:
                break
            steps += 1
        lconv += int(inf_["converged"])
        lits.append(steps)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t
    loop_rate = lconv / t_loop
    log(f"loop: {min(n_loop, n_inst)} instances, {lconv} converged in {t_loop:.2f} s ({loop_rate:.1f} solves/s)")
    return {"workload": f"{n_inst} instances of the 16384-element P2 Euler problem, pool n in (10,20,30) x m in "
                        f"(5,10), EQ sets U(200..2000) + 64 inflow elements, mu Sobol on [2,3] x [-5,5] deg",
            "instances": n_inst, "sum_n_s": ns, "lambda": BATCH_LAMBDA, "max_it": BATCH_MAX_IT, "tol": 1e-8,
            "elements_per_wave": E,
            "solves_per_s": conv / t_solve, "converged": conv, "seconds": t_solve,
            "status_counts": {int(k): int(v) for k, v in zip(st, cnt)},
            "mean_gn_iterations": float(o["iterations"].mean()),
            "jacobian_evals_per_s": ns / t_jac, "jacobian_ms": t_jac * 1e3,
            "roofline_jacobian_phase": roof2,
            "loop": {"instances": min(n_loop, n_inst), "converged": lconv, "seconds": t_loop,
                     "solves_per_s": loop_rate, "mean_gn_iterations": float(np.mean(lits))},
            "speedup_vs_loop": (conv / t_solve) / loop_rate if loop_rate > 0 else None,
            "with_w_only_initialisation": presolve,
            "greedy_indicator": greedy,
            "mixed_precision": mixed}


def batch_jacobian_only(dev, n_inst: int, reps: int = 3):
    """The batched Jacobian phase alone (FP64, then mixed precision) on the
    batched workload at the plain start, each batch autotuned: what a
    profiler run of the batched kernels needs."""
    import torch
    import synth
    from paper_2305_15661_amd import ift
    bw = synth.euler_batch(n_inst=n_inst)
    prob = ift.Problem.from_workload(bw.base)
    pool = [(torch.tensor(np.ascontiguousarray(P), device=dev), torch.tensor(np.ascontiguousarray(S), device=dev))
            for P, S in bw.pool]
    mu = torch.tensor(bw.mus, dtype=torch.float64, device=dev)
    out = {"workload": f"{n_inst} instances of the batched P2 Euler workload, Jacobian phase at the plain start"}
    for prec in ("fp64", "mixed"):
        roms = [ift.ROM(prob, *pool[bw.inst_pool[i]], bw.inst_elem[i], bw.inst_rho[i],
                        "mixed" if prec == "mixed" else "fp64") for i in range(n_inst)]
        b = ift.Batch(roms)
        z0 = torch.zeros(b.nz, dtype=torch.float64, device=dev)
        b.plain_start(mu, z0)
        E = b.autotune(mu, z0)
        by, proj, gram = batch_work(bw, n_inst, mixed=prec == "mixed")
        out[prec] = batch_roofline(b, mu, z0, by, proj, gram, reps, mixed=prec == "mixed")
        out[prec]["elements_per_wave"] = E
        log(f"{prec}: " + ", ".join(f"{k} {v:.0f} us" for k, v in out[prec]["kernels_us"].items()))
        del b, roms
    return out


def warm_start_leg(dev, n_train: int = 4096, n_test: int = 1024, train_steps: int = 3000):
    """Learned warm start on the 16384-element ROM (n = 20, m = 10, 819 EQ
    elements): FP64 batched solves at n_train Sobol mu (seed 1005) give the
    targets; the network 2 -> 128 -> 128 -> 30 is trained on the converged
    ones; n_test held-out Sobol mu (seed 1007) are then solved in the
    mixed-precision batched pipeline from the plain start and from the
    network's start (BF16 inference, plain-start fallback)."""
    import torch
    from scipy.stats import qmc
    import synth
    from paper_2305_15661_amd import ift
    wl = synth.euler_p2(n_eval=1)
    prob = ift.Problem.from_workload(wl)
    Phi = torch.tensor(wl.Phi, device=dev)
    Psi = torch.tensor(wl.Psi, device=dev)
    rom64 = ift.ROM(prob, Phi, Psi, wl.eq_elem, wl.eq_rho)
    romm = ift.ROM(prob, Phi, Psi, wl.eq_elem, wl.eq_rho, "mixed")

    def sobol(seed, n):
        s = qmc.Sobol(d=2, scramble=True, seed=seed).random(n)
        return np.stack([2.0 + s[:, 0], -5.0 + 10.0 * s[:, 1]], axis=1)

    def solve(batch, mu, warm_z=None, reps=1):
        mu_t = torch.tensor(mu, device=dev)
        z0 = torch.zeros(batch.nz, dtype=torch.float64, device=dev)
        batch.plain_start(mu_t, z0)
        info = batch.info_buffer(dev)
        out = None
        for rep in range(reps + 1):   # first run captures the graph
            z = (warm_z if warm_z is not None else z0).clone()
            torch.cuda.synchronize()
            t = time.perf_counter()
            batch.solve(mu_t, z, info, lam=BATCH_LAMBDA, max_it=BATCH_MAX_IT, warm=warm_z is not None)
            torch.cuda.synchronize()
            out = (z, ift.Batch.info_array(info), time.perf_counter() - t)
        return out

    t0 = time.perf_counter()
    mu_tr = sobol(1005, n_train)
    btr = ift.Batch([rom64] * n_train)
    ztr, itr, t_gen = solve(btr, mu_tr)
    ok = itr["converged"] == 1
    Z = ztr.reshape(n_train, 30)[torch.tensor(ok, device=dev)]
    M = torch.tensor(mu_tr[ok], device=dev)
    del btr
    log(f"warm start: {int(ok.sum())}/{n_train} training solves converged in {t_gen:.2f} s")
    net = ift.MLP(2, 128, 30, seed=1)
    Zc = Z.cpu().numpy()
    net.set_normalization(mu_tr[ok].mean(0), mu_tr[ok].std(0), Zc.mean(0), np.maximum(Zc.std(0), 1e-12))
    t = time.perf_counter()
    hist = net.train(M, Z, steps=train_steps, lr=1e-3)
    t_train = time.perf_counter() - t
    log(f"warm start: trained {train_steps} steps in {t_train:.2f} s, loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    mu_te = sobol(1007, n_test)
    bte = ift.Batch([romm] * n_test)
    mu_t = torch.tensor(mu_te, device=dev)
    zw = torch.zeros(bte.nz, dtype=torch.float64, device=dev)
    net.predict(mu_t, zw, bf16=True)
    zp_, ip, tp = solve(bte, mu_te)
    zw_, iw, tw = solve(bte, mu_te, warm_z=zw)
    cp, cw = int(ip["converged"].sum()), int(iw["converged"].sum())
    # the plain FP64 single-instance GPU path on the first n_loop held-out mu:
    # rom_gauss_newton_step from the plain start until convergence
    n_loop = 64
    t = time.perf_counter()
    lconv, lits = 0, []
    for mu in mu_te[:n_loop]:
        w = torch.zeros(rom64.n, dtype=torch.float64, device=dev)
        tau = torch.zeros(rom64.m, dtype=torch.float64, device=dev)
        rom64.plain_start(mu, w, tau)
        steps = 0
        while True:
            last = steps == BATCH_MAX_IT
            wc, tc = (w.clone(), tau.clone()) if last else (w, tau)
            st_, inf_ = rom64.gauss_newton_step(mu, wc, tc, lam=BATCH_LAMBDA)
            if inf_["converged"] or st_ != 0 or last:
                break
            steps += 1
        lconv += int(inf_["converged"])
        lits.append(steps)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t
    loop_rate = lconv / t_loop
    cw_rate = cw / tw
    log(f"warm start: FP64 single-instance loop over {n_loop} held-out mu: {lconv} converged, "
        f"{np.mean(lits):.1f} its, {loop_rate:.1f} solves/s; batched mixed + warm is {cw_rate / loop_rate:.1f}x that")
    log(f"warm start: plain {cp} converged, {ip['iterations'].mean():.1f} its, {tp:.3f} s; warm {cw} converged, "
        f"{iw['iterations'].mean():.1f} its, {tw:.3f} s, {int(np.sum(iw['fallback'] == 1))} fallbacks, "
        f"{int(np.sum(iw['fallback'] == 2))} restarts; statuses {dict(zip(*np.unique(iw['status'], return_counts=True)))}")
    return {"workload": "16384-element P2 Euler ROM, n=20, m=10, 819 EQ elements; mu Sobol on [2,3] x [-5,5] deg",
            "train": {"instances": n_train, "converged": int(ok.sum()), "solve_seconds": t_gen,
                      "steps": train_steps, "train_seconds": t_train, "loss_first": float(hist[0]),
                      "loss_last": float(hist[-1])},
            "test_instances": n_test, "pipeline": "batched, mixed precision (BF16 projection) + FP64 refinement",
            "plain": {"converged": cp, "mean_gn_iterations": float(ip["iterations"].mean()), "seconds": tp,
                      "solves_per_s": cp / tp},
            "warm": {"converged": cw, "mean_gn_iterations": float(iw["iterations"].mean()), "seconds": tw,
                     "solves_per_s": cw / tw, "fallbacks": int(np.sum(iw["fallback"] == 1)),
                     "restarts_after_failed_line_search": int(np.sum(iw["fallback"] == 2))},
            "speedup_warm_vs_plain": (cw / tw) / (cp / tp) if cp and tp > 0 else None,
            "fp64_single_instance_loop": {"instances": n_loop, "converged": lconv, "seconds": t_loop,
                                          "solves_per_s": loop_rate, "mean_gn_iterations": float(np.mean(lits))},
            "speedup_vs_fp64_single_instance_loop": cw_rate / loop_rate if loop_rate > 0 else None,
            "setup_seconds": time.perf_counter() - t0}


def eqp_leg(dev, n_train: int = 8):
    """EQ-weight training at the C1 shape: a ROM over all 16384 elements with
    unit weights, its solutions at n_train training parameters (Gauss-Newton
    steps on the device from the plain start), the elemental reduced
    residuals at each converged solution on the device, and the linear
    program of the paper's weight training solved on the host (HiGHS).  The
    constraints of eq. (eqp-con) are stated at ROM-IFT solutions, so a
    training solve that does not converge is counted and left out."""
    import torch
    import synth
    from scipy.stats import qmc
    from paper_2305_15661_amd import eqp, ift
    wl = synth.euler_p2()
    prob = ift.Problem.from_workload(wl)
    Ne = wl.mesh.n_elem
    t = lambda a: torch.tensor(np.ascontiguousarray(a), device=dev)
    rom = ift.ROM(prob, t(wl.Phi), t(wl.Psi), np.arange(Ne, dtype=np.int32), np.ones(Ne))
    sob = qmc.Sobol(d=2, scramble=True, seed=1010).random(n_train)
    mus = np.stack([2.0 + sob[:, 0], -5.0 + 10.0 * sob[:, 1]], axis=1)
    sols, t_solve, conv = [], 0.0, 0
    for mu in mus:
        w = torch.zeros(rom.n, dtype=torch.float64, device=dev)
        tau = torch.zeros(rom.m, dtype=torch.float64, device=dev)
        rom.plain_start(mu, w, tau)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(BATCH_MAX_IT):
            st, info = rom.gauss_newton_step(mu, w, tau, lam=BATCH_LAMBDA)
            if info["converged"] or st != 0:
                break
        torch.cuda.synchronize()
        t_solve += time.perf_counter() - t0
        conv += int(info["converged"])
        if info["converged"]:
            sols.append((mu, w, tau))
    if not sols:
        log(f"eq training: none of {n_train} training solves converged; program skipped")
        return {"training_solves_converged": 0, "training_solves": n_train}
    C = torch.zeros(Ne * rom.D, dtype=torch.float64, device=dev)
    contribs = []
    rom.element_contributions(sols[0][0], sols[0][1], sols[0][2], C)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for mu, w, tau in sols:
        rom.element_contributions(mu, w, tau, C)
        contribs.append(C.cpu().numpy().reshape(Ne, rom.D).copy())
    t_contrib = time.perf_counter() - t0
    vol = eqp.element_volumes(wl.mesh.X, wl.mesh.elem_gnodes)
    # accuracy tolerance relative to the elemental residuals (their sum, the
    # reduced residual at a solution, is near zero); volume within 1 %
    scale = max(float(np.abs(Cj).max()) for Cj in contribs)
    delta = 1e-3 * scale
    t0 = time.perf_counter()
    rho, info = eqp.train_weights(contribs, vol, delta, delta_vol=1e-2)
    t_lp = time.perf_counter() - t0
    frac = info.get("nnz", Ne) / Ne
    log(f"eq training: {conv}/{n_train} training solves in {t_solve:.2f} s; elemental residuals of {Ne} elements "
        f"x {len(sols)} converged solutions in {t_contrib * 1e3:.1f} ms (incl. copies); program "
        f"{2 + 2 * len(sols) * rom.D} x {Ne} "
        f"solved in {t_lp:.2f} s: {info.get('nnz')} non-zero weights ({100 * frac:.2f} %)")
    return {"workload": f"ROM over all {Ne} P2 Euler elements, n=20, m=10, unit weights; {n_train} training "
                        f"parameters (Sobol on [2,3] x [-5,5] deg)",
            "training_solves": n_train, "training_solves_converged": conv, "training_solve_seconds": t_solve,
            "contribution_seconds": t_contrib, "program_rows": 2 + 2 * len(sols) * rom.D, "program_cols": Ne,
            "delta": delta, "lp_seconds": t_lp, "lp_status": info.get("status"), "nonzero_weights": info.get("nnz"),
            "nonzero_fraction": frac, "max_violation": info.get("max_violation")}


def burgers_leg(dev, reps: int = 50):
    """The space-time Burgers problem of Section 4.1 with its source, at the
    paper's size: 860 P1 elements (43 x 10 cells of (0, 100) x (0, 50)),
    n = m = 3, 52 EQ elements (6 %), and the 7 x 7 test grid of mu = (a, b)
    on [3, 9] x [0.02, 0.075].  EQ Jacobians of all 49 points in one batched
    call, the full-order assembly with Jacobians, and the 49 solves in one
    batch from the plain start.  The synthetic bases leave objectives of
    1e2..1e5 (no basis state solves the problem), where the rounding of the
    objective decides the line search once the gradient norm is down to a
    few 1e-4, so the solves run to a gradient tolerance of 1e-3."""
    import torch
    import synth
    from paper_2305_15661_amd import ift
    wl = synth.spacetime_burgers(n_eval=1, nx=43, ny=10, p=1, n=3, m=3, n_s=52)
    prob = ift.Problem.from_workload(wl)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    rom = ift.ROM(prob, t(wl.Phi), t(wl.Psi), wl.eq_elem, wl.eq_rho)
    ga, gb = np.meshgrid(np.linspace(3.0, 9.0, 7), np.linspace(0.02, 0.075, 7), indexing="ij")
    mus = np.stack([ga.ravel(), gb.ravel()], axis=1)
    P, n, D = len(mus), rom.n, rom.D
    batch = ift.Batch([rom] * P)
    MU = t(mus)
    z0 = torch.zeros(batch.nz, dtype=torch.float64, device=dev)
    batch.plain_start(MU, z0)
    zs = batch.unpack(z0)
    W, T = t(np.stack([z[:n] for z in zs])), t(np.stack([z[n:] for z in zs]))
    rom.reserve(P)
    J, G, H = (torch.zeros(P * k, dtype=torch.float64, device=dev) for k in (1, D, D * D))
    nb = torch.zeros(P, dtype=torch.int32, device=dev)

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_jac = timed(lambda: rom.eq_assemble_jacobian_batch(MU, W, T, J, G, H, nb))
    Ne = wl.mesh.n_elem
    U = t(wl.Phi @ zs[P // 2][:n])
    x = t(wl.X + wl.Psi @ zs[P // 2][n:])
    z = lambda k: torch.zeros(k, dtype=torch.float64, device=dev)
    out = dict(R=z(prob.N_u), N=z(Ne), n_bad=torch.zeros(1, dtype=torch.int32, device=dev),
               dRdU=z(Ne * prob.nue * prob.nue), dRdUn=z(Ne * prob.nue * prob.nun), dRdx=z(Ne * prob.nue * prob.nxe),
               dNdx=z(Ne * prob.nxe))
    t_hdm = timed(lambda: prob.hdm_assemble(mus[P // 2], U, x, **out))
    info = batch.info_buffer(dev)
    zz = z0.clone()
    batch.solve(MU, zz, info, lam=BATCH_LAMBDA, max_it=300, tol=1e-3)
    torch.cuda.synchronize()
    zz = z0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.solve(MU, zz, info, lam=BATCH_LAMBDA, max_it=300, tol=1e-3)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    o = ift.Batch.info_array(info)
    conv = int(o["converged"].sum())
    log(f"space-time Burgers with source: eq jacobian {P} points x {rom.n_s} elements in {t_jac * 1e6:.1f} us "
        f"({P * rom.n_s / t_jac:.3e} evals/s); hdm_assemble {Ne} elements with jacobians {t_hdm * 1e6:.1f} us; "
        f"{conv}/{P} solves converged in {t_solve * 1e3:.2f} ms, mean iterations {o['iterations'].mean():.1f}")
    return {"workload": "space-time Burgers with source s = 0.02 exp(b x), 860 P1 elements (43x10 cells of "
                        "(0,100)x(0,50)), n=3, m=3, 52 EQ elements, 7x7 grid of mu on [3,9]x[0.02,0.075]",
            "eq_jacobian_us": t_jac * 1e6, "eq_jacobian_evals_per_s": P * rom.n_s / t_jac,
            "hdm_assemble_jacobians_us": t_hdm * 1e6, "hdm_evals_per_s": Ne / t_hdm,
            "solves": P, "converged": conv, "solve_seconds": t_solve, "solves_per_s": conv / t_solve,
            "mean_gn_iterations": float(o["iterations"].mean()), "tol": 1e-3, "max_it": 300,
            "status_counts": {str(int(k)): int(v) for k, v in zip(*np.unique(o["status"], return_counts=True))}}


def align_leg(dev, nx: int = 32, ny: int = 16, j: int = 4, steps: int = 3):
    """Snapshot alignment of the greedy loop, eq. (align0), on an nx x ny P2
    Euler mesh: Gauss-Newton on (w, x) with the first j state modes and the
    whole node vector, full-order residual and Jacobian blocks on the device
    (hdm_assemble), sparse normal equations on the host, device line search;
    then the Gram-Schmidt append of x* - X to the mapping basis."""
    import synth
    from paper_2305_15661_amd import align, ift
    wl = synth.euler_p2(nx=nx, ny=ny, n=20, m=10, n_s=12, n_eval=2)
    prob = ift.Problem.from_workload(wl)
    Phi_j = np.linalg.qr(wl.Phi[:, :j])[0]
    al = align.Alignment(prob, Phi_j)
    mu = wl.mus[1]
    w = Phi_j.T @ (wl.Phi @ wl.w_eval[1])
    x = wl.X + wl.Psi @ wl.tau_eval[1]
    al.jacobian(mu, w, x)                       # warm-up
    t0 = time.perf_counter()
    for _ in range(3):
        al.jacobian(mu, w, x)
    t_jac = (time.perf_counter() - t0) / 3
    hist = []
    t0 = time.perf_counter()
    for _ in range(steps):
        w, x, info = al.step(mu, w, x, 1e-2)
        hist.append(info)
    t_steps = (time.perf_counter() - t0) / steps
    Psi1 = align.gram_schmidt_append(np.linalg.qr(wl.Psi)[0], x - wl.X)
    log(f"alignment: {wl.mesh.n_elem} P2 elements, {x.size} node coordinates + {j} state modes: "
        f"device blocks + host assembly {t_jac * 1e3:.1f} ms, {t_steps * 1e3:.1f} ms per step; "
        f"objective {hist[0]['J_old']:.3e} -> {hist[-1]['J_new']:.3e}")
    return {"workload": f"Euler P2 {nx}x{ny} cells ({wl.mesh.n_elem} elements), {x.size} node coordinates, "
                        f"{j} state modes, lambda 1e-2",
            "jacobian_assembly_ms": t_jac * 1e3, "step_ms": t_steps * 1e3, "steps": steps,
            "objective_first": hist[0]["J_old"], "objective_last": hist[-1]["J_new"],
            "statuses": [h["status"] for h in hist], "mapping_basis_columns": int(Psi1.shape[1])}


def _finite(o):
    """The result with every non-finite float (an invalid candidate's norm)
    replaced by None, so that the line is strict JSON."""
    if isinstance(o, dict):
        return {k: _finite(v) for k, v in o.items()}
    if isinstance(o, (list, tuple)):
        return [_finite(v) for v in o]
    if isinstance(o, float) and not math.isfinite(o):
        return None
    return o


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-full", action="store_true",
                    help="the oracle also on a C1 solve and on batched instances one by one (minutes)")
    ap.add_argument("--batch-jacobian-only", action="store_true",
                    help="only the batched Jacobian phase (FP64 and mixed precision), for profilers")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-solve", action="store_true", help="skip the solves/s leg")
    ap.add_argument("--no-hdm", action="store_true", help="skip the full-order leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-solve leg")
    ap.add_argument("--batch-inst", type=int, default=1024, help="instances of the batched-solve leg")
    ap.add_argument("--batch-loop", type=int, default=64, help="instances timed in the per-instance loop")
    ap.add_argument("--no-warm", action="store_true", help="skip the learned warm-start leg")
    ap.add_argument("--no-eqp", action="store_true", help="skip the EQ-weight training leg")
    ap.add_argument("--no-burgers", action="store_true", help="skip the space-time Burgers leg")
    ap.add_argument("--no-align", action="store_true", help="skip the snapshot-alignment leg")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a device copy of this size (traffic-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the library runs one GPU per process; instances shard across GPUs without communication)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")

    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 8 * n, "launches": 5}))
        return

    import synth
    from paper_2305_15661_amd import ift

    if args.batch_jacobian_only:
        print(json.dumps(_finite(batch_jacobian_only(dev, args.batch_inst)), allow_nan=False))
        return

    t_setup = time.perf_counter()
    wl = synth.euler_p2()
    prob = ift.Problem.from_workload(wl)
    Phi = torch.tensor(wl.Phi, device=dev)
    Psi = torch.tensor(wl.Psi, device=dev)
    rom = ift.ROM(prob, Phi, Psi, wl.eq_elem, wl.eq_rho)
    del Phi, Psi
    D, n = rom.D, rom.n
    W = torch.tensor(wl.w_eval, device=dev)
    T = torch.tensor(wl.tau_eval, device=dev)
    J = torch.zeros(1, dtype=torch.float64, device=dev)
    g = torch.zeros(D, dtype=torch.float64, device=dev)
    H = torch.zeros(D * D, dtype=torch.float64, device=dev)
    n_eval = wl.mus.shape[0]
    log(f"setup {time.perf_counter() - t_setup:.1f}s: {wl.mesh.n_elem} elements, n_s={wl.n_s}, n={n}, m={rom.m}")

    # ---------------------------------------------------------- timed steps
    P = n_eval
    rom.reserve(P)
    mu2 = np.zeros((P, 2))
    mu2[:, :wl.mus.shape[1]] = wl.mus
    MU = torch.tensor(mu2, device=dev)
    JB = torch.zeros(P, dtype=torch.float64, device=dev)
    GB = torch.zeros(P * D, dtype=torch.float64, device=dev)
    HB = torch.zeros(P * D * D, dtype=torch.float64, device=dev)
    for s in range(args.warmup):
        rom.eq_assemble_jacobian_batch(MU, W, T, JB, GB, HB)
    torch.cuda.synchronize()
    ift.profile_enable(True)
    ift.profile_reset()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    t0 = time.perf_counter()
    for s in range(args.steps):
        rom.eq_assemble_jacobian_batch(MU, W, T, JB, GB, HB)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ift.profile_enable(False)
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = max(gpu_ms, 1e3 * wall) / args.steps
    evals_per_step = P * wl.n_s
    value = evals_per_step / (ms_per_step * 1e-3)
    kt = {k: ift.profile_read(k) for k in ("points", "eq_jac", "gram")}
    avg = {k: (ms / c * 1e-3 if c else 0.0) for k, (c, ms) in kt.items()}
    log("step %.1f us: " % (ms_per_step * 1e3) + ", ".join(
        f"{k} {v * 1e6:.1f} us x {kt[k][0] / args.steps:.0f}" for k, v in avg.items()))
    # per launch: a kernel may run as several launches per step
    launches = {k: c / args.steps for k, (c, ms) in kt.items()}
    dom = max(avg, key=lambda k: avg[k] * launches[k])
    t_dom = avg[dom]
    units = evals_per_step / launches[dom]          # element-evals per launch
    gbs = KBYTES[dom] * units / t_dom / 1e9
    if KFLOPS[dom] is None:
        roofline = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS}
    else:
        tf = KFLOPS[dom] * units / t_dom / 1e12
        roofline = {"bound": "mfma", "achieved": tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                    "frac": tf / PEAK_FP64_TFLOPS}
    tr = TRAFFIC_KIB.get(dom)
    traffic = None if tr is None else FETCH_SCALE * tr[0] * 1024 + WRITE_SCALE * tr[1] * 1024
    roofline.update({"traffic": traffic, "traffic_source": TRAFFIC_SOURCE if traffic else None,
                     "kernel": KNAMES[dom], "launch_avg_us": t_dom * 1e6,
                     "launches_per_step": launches[dom], "element_evals_per_launch": units,
                     "algorithmic_bytes_per_launch": KBYTES[dom] * units,
                     "algorithmic_flops_per_launch": (KFLOPS[dom] or 0) * units,
                     "kernels_us": {k: v * 1e6 for k, v in avg.items()},
                     "launches_per_step_by_kernel": launches})
    out = {"metric": METRIC, "value": value, "unit": "element-evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "euler_p2 128x64 cells (16384 P2 elements), n=20, m=10, 819 EQ elements, "
                                  "16 evaluation points per step",
                      "n_s": int(wl.n_s), "n": n, "m": int(rom.m), "n_elem": int(wl.mesh.n_elem), "points": P},
           "roofline": roofline}

    # ------------------------------------------------------------- solves/s
    if not args.no_solve:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        conv, iters = 0, []
        for k in range(n_eval):
            w = W[k].clone()
            tau = T[k].clone()
            for it in range(60):
                st, info = rom.gauss_newton_step(wl.mus[k], w, tau)
                if info["converged"] or st != 0:
                    break
            conv += int(info["converged"] == 1)
            iters.append(it)
        dt = time.perf_counter() - t0
        out["solves_per_s"] = conv / dt
        out["solves"] = {"converged": conv, "attempted": n_eval, "mean_gn_iterations": float(np.mean(iters)),
                         "tol": 1e-8, "seconds": dt}
        log(f"solves: {conv}/{n_eval} converged, {conv / dt:.1f} solves/s, mean iterations {np.mean(iters):.1f}")
        # the same solves as one batch (one ROM, the points as instances)
        bs = ift.Batch([rom] * n_eval)
        mub = np.zeros((n_eval, 2))
        mub[:, :wl.mus.shape[1]] = wl.mus[:n_eval]
        mub = torch.tensor(mub, device=dev)
        zb0 = bs.pack([np.r_[W[k].cpu().numpy(), T[k].cpu().numpy()] for k in range(n_eval)], dev)
        infob = bs.info_buffer(dev)
        for rep in range(2):   # the first call captures the graph
            zb = zb0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bs.solve(mub, zb, infob, lam=0.0, max_it=60)
            torch.cuda.synchronize()
            dtb = time.perf_counter() - t0
        ob = ift.Batch.info_array(infob)
        convb = int(ob["converged"].sum())
        out["solves"]["batched"] = {"converged": convb, "seconds": dtb, "solves_per_s": convb / dtb,
                                    "mean_gn_iterations": float(ob["iterations"].mean())}
        log(f"solves as one batch: {convb}/{n_eval} converged, {convb / dtb:.1f} solves/s")
        del bs

    # ------------------------------------------------------- batched solves
    if not args.no_batch:
        out["batched"] = batched_leg(args.batch_inst, args.batch_loop, dev)

    if not args.no_eqp:
        out["eq_training"] = eqp_leg(dev)
    if not args.no_burgers:
        out["spacetime_burgers"] = burgers_leg(dev)
    if not args.no_align:
        out["snapshot_alignment"] = align_leg(dev)
    if not args.no_warm:
        out["warm_start"] = warm_start_leg(dev)

    # ---------------------------------------------------------- full order
    if not args.no_hdm:
        p = prob
        Ne = p.n_elem
        U = torch.tensor(wl.Phi @ wl.w_eval[0], device=dev)
        x = torch.tensor(wl.X + wl.Psi @ wl.tau_eval[0], device=dev)
        R = torch.empty(p.N_u, dtype=torch.float64, device=dev)
        Nn = torch.empty(Ne, dtype=torch.float64, device=dev)
        dRdU = torch.empty(Ne * p.nue * p.nue, dtype=torch.float64, device=dev)
        dRdUn = torch.empty(Ne * p.nue * p.nun, dtype=torch.float64, device=dev)
        dRdx = torch.empty(Ne * p.nue * p.nxe, dtype=torch.float64, device=dev)
        dNdx = torch.empty(Ne * p.nxe, dtype=torch.float64, device=dev)
        for _ in range(3):
            p.hdm_assemble(wl.mus[0], U, x, R, Nn, dRdU, dRdUn, dRdx, dNdx)
        torch.cuda.synchronize()
        ift.profile_enable(True)
        ift.profile_reset()
        reps = 10
        for _ in range(reps):
            p.hdm_assemble(wl.mus[0], U, x, R, Nn, dRdU, dRdUn, dRdx, dNdx)
        torch.cuda.synchronize()
        ift.profile_enable(False)
        c, ms = ift.profile_read("hdm")
        c2, ms2 = ift.profile_read("points")
        t_avg = (ms + ms2) / c * 1e-3
        gbs = HDM_BYTES_PER_ELEM * Ne / t_avg / 1e9
        hdm_traffic = FETCH_SCALE * HDM_TRAFFIC_KIB[0] * 1024 + WRITE_SCALE * HDM_TRAFFIC_KIB[1] * 1024
        out["hdm_assemble"] = {"evals_per_s": Ne / t_avg, "launch_avg_us": t_avg * 1e6, "bound": "hbm",
                               "achieved_GBs": gbs, "frac": gbs / PEAK_HBM_GBS,
                               "traffic": hdm_traffic, "traffic_GBs": hdm_traffic / t_avg / 1e9,
                               "traffic_source": "profiles/hdm_assemble_euler_p2_16384.md",
                               "points_us": ms2 / c2 * 1e3 if c2 else None, "assembly_us": ms / c * 1e3,
                               "kernels": "one pass (point physics and blocks)" if not c2 else "points + assembly"}
        log(f"hdm_assemble: {t_avg * 1e6:.1f} us, {Ne / t_avg:.3e} evals/s, {gbs:.0f} GB/s")
        del dRdU, dRdUn, dRdx

    # ------------------------------------------------------------ CPU leg
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds, args.cpu_full)
        log(f"cpu baseline: {out['cpu_baseline']['value']:.1f} evals/s")
    print(json.dumps(_finite(out), allow_nan=False))


if __name__ == "__main__":
    main()
