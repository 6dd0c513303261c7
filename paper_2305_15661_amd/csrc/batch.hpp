// Batched ROM Gauss-Newton solves: many instances (own mu, own ROM and EQ
// set) advance together on the device, each through the Levenberg-Marquardt
// step and Armijo backtracking of the single-instance solver.
//
// Every instance carries a small state machine (BatchState):
//   BS_JAC     needs the Jacobian assembly at its iterate z,
//   BS_VERIFY  has taken the full step z <- z + dz (the previous iterate
//              kept in zt) and needs the Jacobian assembly there, whose
//              objective decides the Armijo test at alpha = 1,
//   BS_SEARCH  backtracks: tries z + alpha dz, alpha = 1/2, 1/4, ...,
//   BS_DONE    converged or stopped (status says why).
// The full step is taken before its test because nearly every accepted
// step has alpha = 1: the assembly at the new iterate then serves both the
// test and the next step, and a rejected full step only restores z.
// Every Armijo test compares two objectives summed by the same kernels in
// the same order: the full step's test compares the Gram corners of two
// Jacobian assemblies, and backtracking first re-evaluates J~(z) with the
// residual kernels that evaluate its trials (their per-element sums differ
// from the Gram corner's by rounding, which near a minimum is as large as
// the decrease the test asks for).
// Each phase starts with k_batch_compact, which scans the instances in the
// phase's state into work lists (exclusive sums of their element or block
// counts); the work kernels are persistent grids that walk those lists, so
// finished instances cost nothing and uneven EQ sets need no padding.  A
// round (Jacobian phase, LM step, a few line-search trials) is the same
// launch sequence for any state, which lets the host capture a few rounds
// once in a HIP graph and replay them until every instance has finished.
#pragma once
#include "kernels.hpp"

namespace ift {

enum { BS_JAC = 0, BS_SEARCH = 1, BS_DONE = 2, BS_VERIFY = 3 };

// One instance: its ROM's element data and its slices of the batch
// workspace.  a.w / a.tau point at the current iterate z, a.mu at its mu.
struct BatchInst {
  EqArgs a;
  const double* Bw;
  const double* Bx;
  double* z;          // [D]
  double* zt;         // [D] trial iterate
  double* dz;         // [D]
  double* zp;         // [D] plain start kept for a restart (warm-started solves)
  double* H;          // [D * D]
  double* g;          // [D]
  double* part;       // fused partials [nblk][NH][256]
  int* part_bad;      // [nblk][2]
  const double* phisum;  // [n_c][n] column sums of Phi per component (plain start)
  const short* Bw16;  // BF16 point bases (mixed-precision instances), else null
  const short* Bx16;
  int nblk;           // fused blocks of this instance
  int nt;             // fused column tiles (1..FUSED_MAXNT)
};

struct BatchState {
  int state, it, n_bt, status;
  int flag_or, n_bad, converged, n_bt_total;
  int prec;           // 1: mixed-precision rounds, 0: FP64 rounds
  int fallback;       // warm start replaced by the plain start
  int it_mixed;       // LM steps taken in mixed-precision rounds
  int restart;        // 1: a failed line search restarts from the plain start zp
  int prec0;          // precision phase of a fresh start
  int wonly;          // 1: initialisation steps in w with tau held
  int it_w;           // steps taken in w only
  int reval;          // 1: the next trial re-evaluates J~ at z itself (alpha = 0)
  double lam;         // LM weight of the next step
  double J, J0, Jtrial, alpha, slope, nS, nT, alpha_acc;
  double Jprev;       // objective at the previous iterate (BS_VERIFY)
};

struct BatchParams {
  double lambda, c1, tol;
  double tol_mix;     // gradient norms at which a mixed-precision instance switches to FP64
  int max_backtrack, max_it;
  int max_bt_mixed;   // halvings after which a mixed-precision instance switches to FP64
  int adapt;          // 1: lambda / 10 after a full step, max(10 lambda, 1e-8) after a shortened one
};

// Work lists of one phase.  off[q][i] = sum over active instances j < i of
// their count in list q (q = 0: sampled elements; q = t: fused blocks of
// the instances with t column tiles); cnt[q] = the totals.
struct BatchLists {
  int* off;   // [4][n_inst + 1]
  int* cnt;   // [4]
};

// Owner of `item` given the owner h of an earlier item of the same list:
// probes h + 1, h + 2, h + 4, ... upwards, then bisects the bracket.
IFT_DEV int batch_owner_from(const int* off, int n_inst, int item, int h) {
  if (off[h + 1] > item) return h;
  int lo = h + 1, hi = n_inst, step = 1;   // off[lo] <= item < off[hi]
  while (lo + step < n_inst) {
    if (off[lo + step] > item) {
      hi = lo + step;
      break;
    }
    lo += step;
    step <<= 1;
  }
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= item) lo = mid;
    else hi = mid;
  }
  return lo;
}

constexpr int BC_THR = 1024;

// Exclusive sums of the element and block counts of the instances in state
// `want` (and, if want_prec >= 0, in that precision phase); one block,
// fixed order.  with_blocks = 0 leaves the block lists empty.
// (The Jacobian phase, want = BS_JAC, also takes the BS_VERIFY instances.)
IFT_DEV bool batch_active(const BatchState& st, int want, int want_prec) {
  const bool in = st.state == want || (want == BS_JAC && st.state == BS_VERIFY);
  return in && (want_prec < 0 || st.prec == want_prec);
}

__global__ __launch_bounds__(BC_THR) void k_batch_compact(const BatchInst* I, const BatchState* S, BatchLists L,
                                                          int n_inst, int want, int want_prec, int with_blocks) {
  __shared__ int sc[4][BC_THR];
  const int t = threadIdx.x;
  const int chunk = (n_inst + BC_THR - 1) / BC_THR;
  const int beg = min(n_inst, t * chunk), end = min(n_inst, beg + chunk);
  int c[4] = {0, 0, 0, 0};
  for (int i = beg; i < end; ++i) {
    if (!batch_active(S[i], want, want_prec)) continue;
    c[0] += I[i].a.n_s;
    if (with_blocks) c[I[i].nt] += I[i].nblk;
  }
  for (int q = 0; q < 4; ++q) sc[q][t] = c[q];
  __syncthreads();
  // inclusive scan over the threads (Hillis-Steele)
  for (int d = 1; d < BC_THR; d <<= 1) {
    int v[4];
    for (int q = 0; q < 4; ++q) v[q] = t >= d ? sc[q][t - d] : 0;
    __syncthreads();
    for (int q = 0; q < 4; ++q) sc[q][t] += v[q];
    __syncthreads();
  }
  int run[4];
  for (int q = 0; q < 4; ++q) run[q] = sc[q][t] - c[q];
  for (int i = beg; i < end; ++i) {
    const bool act = batch_active(S[i], want, want_prec);
    for (int q = 0; q < 4; ++q) L.off[q * (n_inst + 1) + i] = run[q];
    if (act) {
      run[0] += I[i].a.n_s;
      if (with_blocks) run[I[i].nt] += I[i].nblk;
    }
  }
  if (t == BC_THR - 1)
    for (int q = 0; q < 4; ++q) {
      L.off[q * (n_inst + 1) + n_inst] = sc[q][t];
      L.cnt[q] = sc[q][t];
    }
}

// Point physics of every sampled element of the JAC instances.
// (At least two waves per SIMD: the tangent point physics sits just above
// the register budget of that occupancy once inside the persistent loop.)
template <class D, class R>
__global__ __launch_bounds__(NTHR_PTS, 2) void k_points_batch(const BatchInst* I, BatchLists L, int n_inst) {
  __shared__ ElemLDS<D, R> s;
  const int total = L.cnt[0];
  int inst = 0;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    inst = __builtin_amdgcn_readfirstlane(batch_owner_from(L.off, n_inst, item, inst));
    const int k = item - L.off[inst];
    int tid_i = threadIdx.x;   // formed again per item (kept live across the loop, the task indices spill)
    asm volatile("" : "+v"(tid_i));
    points_eq_body<D, R, true>(s, I[inst].a, k, 0, tid_i);
    __syncthreads();
  }
}

// The same with two listed items per 256-thread block (four-component P2,
// phase_points_pair); the two may belong to different instances, so each
// half keeps its physical constants in LDS.  An odd item count leaves the
// last block one item, computed twice and written once.  (FP32: three
// waves per SIMD, the budget its physics fits.)
template <class D, class R>
__global__ __launch_bounds__(2 * NTHR_PTS, sizeof(R) == 4 ? 3 : 2) void k_points_batch2(const BatchInst* I, BatchLists L, int n_inst) {
  __shared__ ElemLDS<D, R> s[2];
  __shared__ PhysConst spc[2];
  const int total = L.cnt[0];
  const int tid = threadIdx.x, h = __builtin_amdgcn_readfirstlane(tid / NTHR_PTS);
  int inst = 0;
  load_tab<D, R, NTHR_PTS>(s[h], tid % NTHR_PTS);   // constant: visible after the first barrier
  for (int i0 = 2 * blockIdx.x; i0 < total; i0 += 2 * gridDim.x) {
    // The lane's task indices are formed again for each item from an opaque
    // copy of the thread index: kept live across the loop they spill.
    int tid_i = tid;
    asm volatile("" : "+v"(tid_i));
    const int t = tid_i % NTHR_PTS;
    const int item = i0 + min(h, total - 1 - i0);
    inst = __builtin_amdgcn_readfirstlane(batch_owner_from(L.off, n_inst, item, inst));
    const int k = item - L.off[inst];
    const EqArgs& a = I[inst].a;
    if (t == 0) spc[h] = a.mu ? phys_from_mu(a.pc, D::PDE, a.bc_mu_scale, a.mu) : a.pc;
    load_eq<D, R>(s[h], a, k, 0, t);   // ends with a barrier
    phase_points_pair<D, R>(s, tid_i, [&](int e) -> const PhysConst& { return spc[e]; }, R(a.eps));
    __syncthreads();
    phase_distortion_eq<D, R>(s[h], a, k, t);
    if (item == i0 + h) copy_pts<D, R, NTHR_PTS>(reinterpret_cast<Pts<D, R>*>(a.pts) + k, &s[h].p, t);
    __syncthreads();
  }
}

// Fused assembly + Gram of the JAC instances with NT column tiles.
template <class D, class R, int NT>
__global__ __launch_bounds__(NTHR, (fused_blocks_per_cu<D, NT>())) void k_fused_batch(const BatchInst* I, BatchLists L, int n_inst, int E) {
  __shared__ FusedShared<D, R, NT> sh;
  fused_load_tab<D, R, NT>(sh, threadIdx.x);
  const int* off = L.off + NT * (n_inst + 1);
  const int total = L.cnt[NT];
  int inst = 0;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    inst = __builtin_amdgcn_readfirstlane(batch_owner_from(off, n_inst, item, inst));
    const int blk = item - off[inst];
    const BatchInst& bi = I[inst];
    FusedArgs f;
    f.E = E;
    f.nblk = bi.nblk;
    f.part = bi.part;
    f.part_bad = bi.part_bad;
    f.rows = 0;
    f.pts2 = 0;
    fused_body<D, R, NT>(sh, bi.a, bi.Bw, bi.Bx, f, blk, 0);
  }
}

// H, g, the objective and the flags of each JAC instance from its partials.
__global__ __launch_bounds__(256) void k_final_batch(const BatchInst* I, BatchState* S) {
  __shared__ double red[GF_GRP][GF_ENT];
  const int inst = blockIdx.y;
  if (S[inst].state != BS_JAC && S[inst].state != BS_VERIFY) return;
  const BatchInst& bi = I[inst];
  const int D1 = bi.a.D + 1;
  const int nbe = (D1 * (D1 + 1) / 2 + GF_ENT - 1) / GF_ENT;
  if ((int)blockIdx.x > nbe) return;
  BatchState& st = S[inst];
  fused_final_body(bi.part, bi.part_bad, bi.nblk, bi.nt, bi.a.D, bi.H, bi.g, &st.J, &st.n_bad, &st.flag_or,
                   blockIdx.x, 0, red);
}

// Line-search failure rules, shared by the test of the full step and the
// trials.  After n_bt halvings a further halving is allowed unless that
// makes more than max_backtrack, or the instance is in mixed-precision
// rounds and has reached their halving limit.
IFT_DEV bool ls_may_halve(const BatchState& st, const BatchParams& p, int n_bt) {
  return n_bt < p.max_backtrack && !(st.prec == 1 && n_bt >= p.max_bt_mixed);
}

// A failed line search that restarts from the plain start (warm starts).
IFT_DEV bool ls_restarts(const BatchState& st, const BatchParams& p) {
  return !st.wonly && !(st.prec == 1 && st.n_bt >= p.max_bt_mixed) && st.restart;
}

// State after a line search that found no decrease within its halvings
// (st.n_bt of them): the w-only initialisation ends, a mixed-precision
// instance continues in FP64 rounds, a warm-started instance restarts from
// the plain start (the caller has copied zp into z), else the solve stops.
IFT_DEV void ls_failed(BatchState& st, const BatchParams& p) {
  const int nb = st.n_bt;
  st.n_bt = nb + 1;
  st.n_bt_total += st.n_bt;
  st.reval = 0;
  if (st.wonly && nb >= p.max_backtrack) {
    st.wonly = 0;       // the initialisation ends here; full steps from this iterate
    st.state = BS_JAC;
  } else if (st.prec == 1 && nb >= p.max_bt_mixed) {
    st.prec = 0;        // no decrease at mixed precision: continue in FP64
    st.state = BS_JAC;
  } else if (st.restart) {
    st.restart = 0;
    st.fallback = 2;
    st.prec = st.prec0;
    st.state = BS_JAC;
  } else {
    st.status = IFT_ELINESEARCH;
    st.state = BS_DONE;
  }
}

// Armijo test of a full step (BS_VERIFY) and then, as for a BS_JAC
// instance, the convergence test and the next LM step (one wave each).
__global__ __launch_bounds__(64) void k_lm_batch(const BatchInst* I, BatchState* S, const BatchParams* P) {
  __shared__ double L[64 * 64];
  __shared__ double y[64];
  __shared__ double out[4];
  __shared__ int fail;
  const int inst = blockIdx.x;
  BatchState& st = S[inst];
  const int state = st.state;
  if (state != BS_JAC && state != BS_VERIFY) return;
  const BatchInst& bi = I[inst];
  const int D = bi.a.D, n = bi.a.n;
  const BatchParams p = *P;
  const double J = st.J;
  double lam = st.lam;
  if (state == BS_VERIFY) {
    // J (+inf if invalid) is the objective at z = z_prev + dz
    const bool ok = J <= st.Jprev + p.c1 * st.slope;
    if (!ok) {
      // restore the previous iterate; the backtracking continues from the
      // first halving, after J~(z) has been re-evaluated by the residual
      // kernels of the trials; with no halving allowed the trial at
      // alpha = 1 has failed for good
      const bool halve = ls_may_halve(st, p, 0);
      const bool restart = !halve && ls_restarts(st, p);
      const double* src = restart ? bi.zp : bi.zt;
      for (int i = threadIdx.x; i < D; i += 64) bi.z[i] = src[i];
      __syncthreads();
      if (threadIdx.x == 0) {
        st.Jtrial = J;
        st.J = st.Jprev;
        if (halve) {
          st.alpha = 0.5;
          st.n_bt = 1;
          st.reval = 1;
          st.state = BS_SEARCH;
        } else {
          st.n_bt = 0;
          ls_failed(st, p);
        }
      }
      return;
    }
    if (p.adapt) lam = lam * 0.1 < 1e-12 ? 0.0 : lam * 0.1;
    if (threadIdx.x == 0) {
      st.Jtrial = J;
      st.alpha_acc = 1.0;
      st.lam = lam;
    }
  }
  if (!(J < __builtin_inf())) {   // invalid geometry or state at the iterate
    if (threadIdx.x == 0) {
      st.status = (st.flag_or & BAD_GEOM) ? IFT_EBADMESH : IFT_ENONPHYS;
      st.state = BS_DONE;
    }
    return;
  }
  // initialisation steps (remark rem:solver): w only, tau held, until
  // |S~| meets the tolerance of the precision phase; then the full step at
  // the same iterate
  const int wonly = st.wonly;
  const int prec = st.prec;
  lm_solve_body(bi.H, bi.g, D, n, wonly ? n : D, lam, bi.dz, out, L, y, fail);
  bool w_step = wonly != 0;
  if (wonly && out[1] <= (prec == 1 ? p.tol_mix : p.tol)) {
    lm_solve_body(bi.H, bi.g, D, n, D, lam, bi.dz, out, L, y, fail);
    w_step = false;
  }
  // the decision below, taken by every lane (all read the same values)
  bool step;
  int next_prec = prec;
  int stop = 0;      // an error status that ends the solve
  bool conv = false;
  if (w_step) {
    if (st.it >= p.max_it) stop = IFT_ENOTCONV;
    else if (out[0] != 0.0) stop = IFT_ESINGULAR;
    step = stop == 0;
  } else if (prec == 1 && out[1] <= p.tol_mix && out[2] <= p.tol_mix) {
    next_prec = 0;   // refine in FP64 from here; the state stays JAC
    step = false;
  } else if (out[1] <= p.tol && out[2] <= p.tol && prec == 0) {
    conv = true;
    step = false;
  } else {
    if (st.it >= p.max_it) stop = IFT_ENOTCONV;
    else if (out[0] != 0.0) stop = IFT_ESINGULAR;
    step = stop == 0;
  }
  __syncthreads();   // every lane has read the state before lane 0 writes it
  if (step)   // keep z in zt and take the full step (same arithmetic as a trial at alpha = 1)
    for (int i = threadIdx.x; i < D; i += 64) {
      const double zi = bi.z[i];
      bi.zt[i] = zi;
      bi.z[i] = zi + 1.0 * bi.dz[i];
    }
  if (threadIdx.x == 0) {
    if (st.it == 0 && prec == 1) st.J0 = J;
    if (st.it == 0 && prec == 0 && st.J0 == 0.0) st.J0 = J;
    st.nS = out[1];
    st.nT = out[2];
    if (!w_step) st.wonly = 0;
    st.prec = next_prec;
    if (conv) {
      st.converged = 1;
      st.status = IFT_OK;
      st.state = BS_DONE;
    } else if (stop != 0) {
      st.status = stop;
      st.state = BS_DONE;
    } else if (step) {
      st.slope = out[3];
      st.Jprev = J;
      st.alpha = 1.0;
      st.n_bt = 0;
      st.it += 1;
      st.it_w += w_step ? 1 : 0;
      st.it_mixed += prec;
      st.state = BS_VERIFY;
    } else {
      st.state = BS_JAC;
    }
  }
}

// Trial iterate z + alpha dz of each SEARCH instance.
__global__ __launch_bounds__(64) void k_trial_batch(const BatchInst* I, const BatchState* S) {
  const int inst = blockIdx.x;
  if (S[inst].state != BS_SEARCH) return;
  const BatchInst& bi = I[inst];
  if (S[inst].reval) {   // J~ at z itself, by the kernels that evaluate the trials
    for (int i = threadIdx.x; i < bi.a.D; i += 64) bi.zt[i] = bi.z[i];
    return;
  }
  const double al = S[inst].alpha;
  for (int i = threadIdx.x; i < bi.a.D; i += 64) bi.zt[i] = bi.z[i] + al * bi.dz[i];
}

// Residual and objective parts at the trial iterates (values only),
// RV_SLOTS elements per block and pass, each lane group on its own item
// (the items of one block may belong to different instances).
template <class D, class R>
__global__ __launch_bounds__(RV_THR) void k_res_batch(const BatchInst* I, BatchLists L, int n_inst) {
  __shared__ ResShared<D, R> sh;
  const int tid = threadIdx.x, g = tid / RV_LANES, j = tid % RV_LANES;
  res_load_tab<D, R>(sh, tid);
  __syncthreads();
  const int total = L.cnt[0];
  int inst = 0;
  for (int base = blockIdx.x * RV_SLOTS; base < total; base += gridDim.x * RV_SLOTS) {
    const int item = base + g;
    const bool act = item < total;
    if (act) inst = batch_owner_from(L.off, n_inst, item, inst);
    const int k = act ? item - L.off[inst] : 0;
    EqArgs a = I[inst].a;
    a.w = I[inst].zt;
    a.tau = I[inst].zt + a.n;
    a.Ft = nullptr;
    a.PTR = nullptr;
    res_group_body<D, R>(sh, sh.e[g], a, k, 0, act, j);
  }
}

// Objective at the trial iterate (fixed-order sum) and the Armijo test.
__global__ __launch_bounds__(256) void k_ls_batch(const BatchInst* I, BatchState* S, const BatchParams* P) {
  __shared__ double sj[256];
  __shared__ int so[256];
  const int inst = blockIdx.x;
  BatchState& st = S[inst];
  if (st.state != BS_SEARCH) return;
  const BatchInst& bi = I[inst];
  const int t = threadIdx.x;
  double v = 0.0;
  int o = 0;
  for (int k = t; k < bi.a.n_s; k += 256) {
    v += bi.a.Jpart[k];
    o |= bi.a.flags[k];
  }
  sj[t] = v;
  so[t] = o;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (t < d) {
      sj[t] += sj[t + d];
      so[t] |= so[t + d];
    }
    __syncthreads();
  }
  const BatchParams p = *P;
  const double Jt = so[0] ? __builtin_inf() : sj[0];
  if (st.reval) {
    // J~(z) by the same kernels and order as the trials; the backtracking
    // continues with the halving already recorded
    __syncthreads();
    if (t == 0) {
      st.J = Jt;
      st.reval = 0;
    }
    return;
  }
  // accept: copy the trial iterate (all lanes), then update the state
  const bool ok = Jt <= st.J + p.c1 * st.alpha * st.slope;
  const bool halve = !ok && ls_may_halve(st, p, st.n_bt);
  const bool restart = !ok && !halve && ls_restarts(st, p);
  if (ok)
    for (int i = t; i < bi.a.D; i += 256) bi.z[i] = bi.zt[i];
  if (restart)
    for (int i = t; i < bi.a.D; i += 256) bi.z[i] = bi.zp[i];
  __syncthreads();
  if (t == 0) {
    st.Jtrial = Jt;
    if (ok) {
      st.alpha_acc = st.alpha;
      st.n_bt_total += st.n_bt;
      st.state = BS_JAC;
      if (p.adapt) {
        if (st.alpha == 1.0) st.lam = st.lam * 0.1 < 1e-12 ? 0.0 : st.lam * 0.1;
        else st.lam = fmax(10.0 * st.lam, 1e-8);
      }
    } else if (halve) {
      st.alpha *= 0.5;
      st.n_bt += 1;
    } else {
      ls_failed(st, p);
    }
  }
}

// Number of instances that have not finished (one block, fixed order).
__global__ __launch_bounds__(256) void k_batch_remaining(const BatchState* S, int n_inst, int* out) {
  __shared__ int sc[256];
  int c = 0;
  for (int i = threadIdx.x; i < n_inst; i += 256) c += S[i].state != BS_DONE;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) sc[threadIdx.x] += sc[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sc[0];
}

// Plain start w0 = Phi^T U_fs(mu_i), tau0 = 0 of every instance into out
// (one block per instance).
__global__ __launch_bounds__(64) void k_plain_batch(const BatchInst* I, int pde, int nc, double* const* outp,
                                                     int which) {
  const int inst = blockIdx.x;
  const BatchInst& bi = I[inst];
  const PhysConst q = phys_from_mu(bi.a.pc, pde, bi.a.bc_mu_scale, bi.a.mu);
  double* out = which == 0 ? bi.z : (which == 1 ? bi.zt : bi.dz);
  (void)outp;
  const int n = bi.a.n, D = bi.a.D;
  for (int j = threadIdx.x; j < D; j += 64) {
    double v = 0.0;
    if (j < n)
      for (int c = 0; c < nc; ++c) v += q.uinf[c] * bi.phisum[c * n + j];
    out[j] = v;
  }
}

// Start selection: stage a candidate start in zt (which 0: the warm start
// z, 1: the plain start held in dz) and mark every instance SEARCH.
__global__ __launch_bounds__(64) void k_start_stage(const BatchInst* I, BatchState* S, int which) {
  const int inst = blockIdx.x;
  const BatchInst& bi = I[inst];
  const double* src = which == 0 ? bi.z : bi.dz;
  for (int j = threadIdx.x; j < bi.a.D; j += 64) bi.zt[j] = src[j];
  if (threadIdx.x == 0) S[inst].state = BS_SEARCH;
}

// Objective at the staged start (fixed-order sum; +inf if invalid) into
// Jtrial (which 0) or alpha (which 1, used as scratch before the solve).
__global__ __launch_bounds__(256) void k_start_obj(const BatchInst* I, BatchState* S, int which) {
  __shared__ double sj[256];
  __shared__ int so[256];
  const int inst = blockIdx.x;
  const BatchInst& bi = I[inst];
  const int t = threadIdx.x;
  double v = 0.0;
  int o = 0;
  for (int k = t; k < bi.a.n_s; k += 256) {
    v += bi.a.Jpart[k];
    o |= bi.a.flags[k];
  }
  sj[t] = v;
  so[t] = o;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (t < d) {
      sj[t] += sj[t + d];
      so[t] |= so[t + d];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double J = so[0] ? __builtin_inf() : sj[0];
    if (which == 0) S[inst].Jtrial = J;
    else S[inst].alpha = J;
  }
}

// Keep the warm start only if its objective is the smaller one.
__global__ __launch_bounds__(64) void k_start_select(const BatchInst* I, BatchState* S) {
  const int inst = blockIdx.x;
  const BatchInst& bi = I[inst];
  BatchState& st = S[inst];
  const bool warm = st.Jtrial < st.alpha;   // false for NaN or +inf warm objectives
  for (int j = threadIdx.x; j < bi.a.D; j += 64) {
    if (warm) bi.zp[j] = bi.dz[j];
    else bi.z[j] = bi.dz[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st.fallback = warm ? 0 : 1;
    st.restart = warm ? 1 : 0;
    st.state = BS_JAC;
    st.Jtrial = 0.0;
    st.alpha = 0.0;
  }
}

// Keeps every stride-th instance in its state and marks the others DONE
// (the autotuner's stand-in for the late rounds of a solve).
__global__ void k_batch_keep_every(BatchState* S, int n_inst, int stride) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_inst && i % stride != 0) S[i].state = BS_DONE;
}

// Fresh state for every instance.
__global__ void k_batch_init(BatchState* S, int n_inst, int mixed, int presolve, double lambda) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_inst) return;
  BatchState st;
  st.state = BS_JAC;
  st.it = 0;
  st.n_bt = 0;
  st.status = IFT_OK;
  st.flag_or = 0;
  st.n_bad = 0;
  st.converged = 0;
  st.n_bt_total = 0;
  st.prec = mixed;
  st.fallback = 0;
  st.it_mixed = 0;
  st.restart = 0;
  st.prec0 = mixed;
  st.wonly = presolve;
  st.it_w = 0;
  st.reval = 0;
  st.lam = lambda;
  st.J = st.J0 = st.Jtrial = 0.0;
  st.alpha = st.slope = st.nS = st.nT = st.alpha_acc = 0.0;
  S[i] = st;
}

}  // namespace ift

