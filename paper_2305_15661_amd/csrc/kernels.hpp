// Kernels of the element loop (full order and EQ-sampled), the deterministic
// reductions, and the small dense solve of the Levenberg-Marquardt step.
//
// Values only (residual, objective): one fused kernel, sixteen lanes per
// element.
// With Jacobians: a point-physics kernel (one thread per quadrature point
// and input direction, tangent arithmetic) writes each element's point
// Jacobians to a workspace; an assembly kernel then builds the explicit
// element Jacobian in LDS and either stores its blocks (full order) or
// projects it onto the gathered reduced bases on FP64 matrix cores (EQ).
#pragma once
#include "element.hpp"

namespace ift {

typedef double dvec4 __attribute__((ext_vector_type(4)));

constexpr int NTHR_PTS = 128;   // point-physics kernel block size

// ---------------------------------------------------------------- arguments
struct HdmArgs {
  const double* U;
  const double* x;
  const int* gn;     // [Ne][nn]
  const int* face;   // [Ne][3]
  const int* Pn;     // [Ne][nun]
  const double* X;   // [N_x]
  double* R;
  double* N;
  double* dRdU;
  double* dRdUn;
  double* dRdx;
  double* dNdx;
  int* flags;        // [Ne]
  void* pts;         // [Ne] point-data workspace
  const double* eta_ref;   // [Ne]: distortion of each reference element
  PhysConst pc;
  double kappa, eps;
  int n_elem;
};

// EQ kernels: blockIdx.x = sampled element k, blockIdx.y = evaluation point.
// Per-point arrays are laid out point-major with the strides below.
struct EqArgs {
  int n_s, n, m, D;
  long long nrows;       // n_s*nue + n_s
  const int* face_s;     // [n_s][3]: face codes of the sampled elements
  const double* rho;     // [n_s]
  const double* srho;    // [n_s] sqrt(rho)
  const double* Phi_s;   // [n_s][nue][n]
  const double* Phin_s;  // [n_s][nun][n]
  const double* Psi_s;   // [n_s][nxe][m]
  const double* X_s;     // [n_s][nxe]
  const double* eta_ref_s;   // [n_s]: distortion of each sampled reference element
  const double* LiftU;   // [n_s][n][nue + nun]: Phi_s then Phin_s rows, column-major per element
  const double* LiftX;   // [n_s][m][nxe]: Psi_s, column-major per element
  const double* w;       // [pt][n]
  const double* tau;     // [pt][m]
  const double* mu;      // [pt][2] on the device, or null: use pc
  const PhysConst* pcs;  // [pt]: the points' physical constants for the point kernels (filled by
                         // k_phys_points from mu), or null: use pc
  double* Jt;            // [pt][nrows][D]
  double* Ft;            // [pt][nrows] (may be null for the residual kernel)
  double* Jpart;         // [pt][n_s]
  int* flags;            // [pt][n_s]
  double* PTR;           // [pt][n_s][n] or null
  void* pts;             // [pt][n_s] point-data workspace
  PhysConst pc;
  double kappa, eps, bc_mu_scale;
};

IFT_DEV PhysConst phys_from_mu(const PhysConst& base, int pde, double bc_scale, const double* mu) {
  PhysConst pc = base;
  if (pde == PDE_BURGERS) {
    pc.uinf[0] = base.bc_st ? mu[0] : 1.0 + bc_scale * mu[0];
    pc.uinf[1] = base.bc_st ? 1.0 : pc.uinf[0];
    pc.src_b = base.src_amp != 0.0 ? mu[1] : 0.0;
  } else {
    const double M = mu[0], a = mu[1] * (M_PI / 180.0), c = sqrt(base.gamma);
    pc.uinf[0] = 1.0;
    double sa, ca;
    sincos(a, &sa, &ca);   // one shared argument reduction
    pc.uinf[1] = M * c * ca;
    pc.uinf[2] = M * c * sa;
    pc.uinf[3] = 1.0 / (base.gamma - 1.0) + 0.5 * base.gamma * M * M;
  }
  return pc;
}

// The physical constants of every evaluation point of a multi-point call,
// once per call: the point kernels then read them with scalar loads instead
// of each block forming them on the vector unit before its physics.
__global__ __launch_bounds__(64) void k_phys_points(PhysConst base, int pde, double bc_scale, const double* mu,
                                                    int n_pts, PhysConst* out) {
  const int p = blockIdx.x * 64 + threadIdx.x;
  if (p < n_pts) out[p] = phys_from_mu(base, pde, bc_scale, mu + 2 * p);
}

// The physical constants of point pt in a point kernel: a.pcs[pt] through
// the constant address space, so that they arrive by scalar loads (as a
// select of pointers the compiler makes it a flat load), else a.pc.
IFT_DEV PhysConst point_consts(const EqArgs& a, int pt) {
  using cpc = const __attribute__((address_space(4))) PhysConst;
  PhysConst pc = a.pc;
  if (a.pcs) {
    cpc* q = (cpc*)a.pcs + pt;
    pc.gamma = q->gamma;
#pragma unroll
    for (int c = 0; c < 4; ++c) pc.uinf[c] = q->uinf[c];
    pc.src_amp = q->src_amp;
    pc.src_b = q->src_b;
    pc.all_farfield = q->all_farfield;
    pc.bc_st = q->bc_st;
  }
  return pc;
}

// Copies one element's point data between LDS (ElemLDS::p, 16-byte aligned)
// and the point workspace, whose element slots start at multiples of the
// FP64 point-data size from a 256-byte aligned base: 16-byte words where
// both sizes are multiples of 16.
template <class D, class R, int NT>
IFT_DEV void copy_pts(Pts<D, R>* dst, const Pts<D, R>* src, int tid) {
  constexpr int A = sizeof(Pts<D, R>) % 16 == 0 && sizeof(Pts<D, double>) % 16 == 0 ? 16 : alignof(Pts<D, R>);
  copy_obj<Pts<D, R>, NT, A>(dst, src, tid);
}

// ------------------------------------------------------------------ loaders
// Direct global-to-LDS loads (gfx950): lane l of the wave moves the 16 bytes
// at src + 16 l to dst + 16 l, for the lanes below nl; dst is the same LDS
// address in every lane.  They count in vmcnt like other vector loads and
// return in order, so "at most N outstanding" means that every load issued
// before the last N has landed.
using lds_void_t = __attribute__((address_space(3))) void;
using gbl_void_t = __attribute__((address_space(1))) void;
IFT_DEV void dma16_at(const void* lane_src, void* dst, bool on) {
  if (on) __builtin_amdgcn_global_load_lds((gbl_void_t*)lane_src, (lds_void_t*)dst, 16, 0, 0);
}
IFT_DEV void dma16(const void* src, void* dst, int lane, int nl) {
  dma16_at(static_cast<const char*>(src) + 16 * lane, dst, lane < nl);
}
// Waits until at most N vector memory loads of the wave are outstanding (a
// compiler memory barrier too, so no LDS read moves above it).
template <int N>
IFT_DEV void vm_wait() {
  static_assert(N >= 0 && N < 16, "vmcnt immediate");
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// acc + sum_j row[j * stride] v[j], accumulated in index order.  The loads
// of a chunk of CH terms are issued together: summed in a plain loop, each
// term would wait for its own load (a cache round trip per basis
// coefficient).  CH trades those round trips against registers.
template <int CH = 16>
IFT_DEV double lift_dot(const double* row, int stride, const double* v, int n, double acc) {
  for (int j0 = 0; j0 < n; j0 += CH) {
    double r[CH], c[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int j = min(j0 + u, n - 1);
      r[u] = row[(long long)j * stride];
      c[u] = v[j];
    }
#pragma unroll
    for (int u = 0; u < CH; ++u)
      if (j0 + u < n) acc += r[u] * c[u];
  }
  return acc;
}

template <class D, class R>
IFT_DEV void load_hdm(ElemLDS<D, R>& s, const HdmArgs& a, int e, int tid, int nthr) {
  constexpr int ntask = D::NUE + D::NUN + 2 * D::NXE + 4;
  for (int k = tid; k < ntask; k += nthr) {
    if (k < D::NUE) {
      s.U[k] = R(a.U[(long long)e * D::NUE + k]);
    } else if (k < D::NUE + D::NUN) {
      int r = k - D::NUE;
      int idx = a.Pn[(long long)e * D::NUN + r];
      s.Un[r] = idx >= 0 ? R(a.U[idx]) : R(0);
    } else if (k < D::NUE + D::NUN + D::NXE) {
      int r = k - D::NUE - D::NUN;
      long long g = a.gn[(long long)e * D::NN + r / 2];
      s.x[r] = R(a.x[2 * g + (r & 1)]);
    } else if (k < D::NUE + D::NUN + 2 * D::NXE) {
      int r = k - D::NUE - D::NUN - D::NXE;
      long long g = a.gn[(long long)e * D::NN + r / 2];
      s.X[r] = R(a.X[2 * g + (r & 1)]);
    } else {
      int f = k - D::NUE - D::NUN - 2 * D::NXE;
      if (f < 3) s.face[f] = a.face[e * 3 + f];
      else s.eta_ref = R(a.eta_ref[e]);
    }
  }
  if (tid == 0) s.p.bad = 0;
}

// Buffer resource over nbytes bytes from p (raw, unswizzled, the untyped
// data format of gfx9); its base and size must be uniform across the wave.
IFT_DEV __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, int nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, nbytes, 0x00020000);
}

// acc = init + sum_j B_j v_j over a column-major block (column j at byte
// offset j * cstride, this lane's entry at lane_bytes within it),
// accumulated in index order; with PAIR the lane holds two adjacent entries
// (16 bytes) and accumulates both from zero, acc2 for the second.  init
// enters after the first chunk's loads issue (a load still in flight there
// costs no wait ahead of them).  Run by a whole wave; only lanes with
// `own` load (the address unit's time goes by active lanes), the others
// compute on whatever their registers hold and must drop the result.  The
// loads of CH columns (CH divides 64) are in flight together, addressed by
// one lane offset shared by all of them and a scalar column offset each.
// In chunks of 32, groups of 8 columns wholly past n are skipped (one
// uniform branch per group); otherwise a column past n reloads column
// n - 1, in bounds, with weight zero, which leaves the sum unchanged.  The coefficients v (n
// <= 64) go through cl, 64 LDS slots of this wave: lane j writes v_j (zero
// from n on) once the first chunk's loads are issued, and the products read
// them back as broadcasts (LDS operations of a wave complete in order).
// during() runs once there too, while those loads are in flight.
struct NoOp {
  IFT_DEV void operator()() const {}
};
template <int CH, bool PAIR = false, class F = NoOp>
IFT_DEV void lift_col_dot(__amdgpu_buffer_rsrc_t B, bool own, int lane_bytes, int cstride, const double* v, double* cl,
                          int n, double init, double& acc, double& acc2, const F& during = F()) {
  static_assert(64 % CH == 0, "chunks tile the 64 coefficient slots");
  const int lane = threadIdx.x & 63;
  acc = 0.0;
  acc2 = 0.0;
  for (int j0 = 0; j0 < n; j0 += CH) {
    constexpr int G = CH > 16 ? 8 : CH;   // (grouping smaller chunks costs the batched kernels registers)
    double r[CH], r2[CH], cc[CH];
    if (own) {
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        if (u % G == 0 && j0 + u >= n) break;
        const int col = min(j0 + u, n - 1);
        if constexpr (PAIR) {
          const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(B, lane_bytes, col * cstride, 0);
          r[u] = __builtin_bit_cast(double, (unsigned long long)q.x | ((unsigned long long)q.y << 32));
          r2[u] = __builtin_bit_cast(double, (unsigned long long)q.z | ((unsigned long long)q.w << 32));
        } else {
          r[u] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(B, lane_bytes, col * cstride, 0));
          r2[u] = 0.0;
        }
      }
    }
    if (j0 == 0) {
      cl[lane] = lane < n ? v[lane] : 0.0;
      during();
    }
    __builtin_amdgcn_sched_barrier(0);   // every load of the chunk issues before the first product
    if (j0 == 0) acc = init;
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      if (u % G == 0 && j0 + u >= n) break;
      cc[u] = cl[j0 + u];
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      if (u % G == 0 && j0 + u >= n) break;
      acc += r[u] * cc[u];
      if constexpr (PAIR) acc2 += r2[u] * cc[u];
    }
  }
  if (n <= 0) {   // no chunk: the hook still runs once
    during();
    acc = init;
  }
}

// Lift U_e = Phi_e w, U_e' = Phi_e' w, x_e = X_e + Psi_e tau for one
// element of NTHR_PTS threads (two waves): one lane per row, a serial dot
// product in index order over the column-major copies of the gathered bases,
// so that the lanes of a wave read adjacent entries of a column.  The first
// wave takes the U rows (two per lane where their count is even: 16-byte
// loads), the second the x rows, the face codes, the reference distortion
// and the flag; every lane of a wave runs the lift (surplus lanes on a
// clamped row; only the rows' own lanes load), so nothing in it waits
// behind a divergent branch, and each wave's loads cost one round trip for
// n <= CH (x rows: m <= 16).  k must be uniform across
// each wave.  Ends with a barrier: everything it wrote is visible to the
// block.
// during() runs in both waves once the lift's first loads are issued (work
// whose own loads then wait beside the lift's, such as the table copy).
template <class D, class R, int CH = 16, class F = NoOp>
IFT_DEV void load_eq(ElemLDS<D, R>& s, const EqArgs& a, int k, int pt, int tid, const F& during = F()) {
  constexpr int RU = D::NUE + D::NUN;
  constexpr bool PAIR = RU % 2 == 0;          // two U rows per lane (16-byte loads)
  constexpr int NU = PAIR ? RU / 2 : RU;      // lanes of the U rows
  static_assert(NTHR_PTS == 128 && NU <= 64 && D::NXE + 4 <= 64, "U rows in the first wave, the rest in the second");
  const int n = a.n, m = a.m;
  const int ku = __builtin_amdgcn_readfirstlane(k);
  const int lane = tid & 63;
  if (tid < 64) {
    const int r0 = PAIR ? 2 * min(lane, NU - 1) : min(lane, NU - 1);
    const auto B = buf_rsrc(a.LiftU + (long long)ku * n * RU, n * RU * 8);
    double acc, acc2;
    lift_col_dot<CH, PAIR>(B, lane < NU, r0 * 8, RU * 8, a.w + (long long)pt * n, s.cf[0], n, 0.0, acc, acc2, during);
    if (lane < NU) {
      if (r0 < D::NUE) s.U[r0] = R(acc);
      else s.Un[r0 - D::NUE] = R(acc);
      if (PAIR) {
        if (r0 + 1 < D::NUE) s.U[r0 + 1] = R(acc2);
        else s.Un[r0 + 1 - D::NUE] = R(acc2);
      }
    }
  } else {
    const int q = min(lane, D::NXE - 1);
    const double X = a.X_s[(long long)ku * D::NXE + q];
    const int fc = a.face_s[ku * 3 + min(max(lane - D::NXE, 0), 2)];
    const double er = a.eta_ref_s[ku];
    const auto B = buf_rsrc(a.LiftX + (long long)ku * m * D::NXE, m * D::NXE * 8);
    double acc, unused;
    lift_col_dot<16>(B, lane < D::NXE, q * 8, D::NXE * 8, a.tau + (long long)pt * m, s.cf[1], m, X, acc, unused,
                     during);
    if (lane < D::NXE) {
      s.x[q] = R(acc);
      s.X[q] = R(X);
    } else if (lane < D::NXE + 3) {
      s.face[lane - D::NXE] = fc;
    } else if (lane == D::NXE + 3) {
      s.p.bad = 0;
      s.eta_ref = R(er);
    }
  }
  __syncthreads();
}

// ------------------------------------------------- full order, values only
template <class D, class R>
__global__ __launch_bounds__(NTHR) void k_hdm_val(HdmArgs a) {
  __shared__ ElemLDS<D, R> s;
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  load_tab<D, R, NTHR>(s, tid);
  load_hdm<D, R>(s, a, e, tid, NTHR);
  __syncthreads();
  phase_points<D, R, false>(s, tid, a.pc, R(a.kappa), R(a.eps));
  __syncthreads();
  phase_assemble<D, R, false>(s, tid);
  __syncthreads();
  if (a.R && tid < D::NUE) a.R[(long long)e * D::NUE + tid] = double(s.Re[tid]);
  if (tid == 0) {
    if (a.N) a.N[e] = double(s.p.N);
    a.flags[e] = s.p.bad;
  }
}

// ------------------------------------------------ point physics (tangent)
// Outputs of one full-order element with four state components, from its
// point data in LDS: R_e, N_e, the flags, dN_e/dx_e and the blocked entries
// of the element Jacobian, written straight to the outputs ((row, node)
// pairs of dR/dU_e and dR/dU_e', four columns each; (row, node) pairs of
// dR/dx_e, two columns).
template <class D, class R>
IFT_DEV void hdm_write_blocks(const ElemLDS<D, R>& s, const HdmArgs& a, int e, int tid, int nthr) {
  static_assert(D::NC == 4, "four state components");
  constexpr int NU = D::NUE * D::NN, NUN4 = D::NUE * 3 * D::NE, NX = D::NUE * D::NN;
  if (a.R && tid < D::NUE) a.R[(long long)e * D::NUE + tid] = double(residual_entry<D, R>(s, tid));
  for (int task = tid; task < NU + NUN4 + NX; task += nthr) {
    R v[4];
    if (task < NU) {
      if (!a.dRdU) continue;
      const int r = task / D::NN, j = task % D::NN;
      jac_u4<D, R>(s.tab, s.p, r, j, v);
      double* o = a.dRdU + ((long long)e * D::NUE + r) * D::NUE + 4 * j;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) o[cc] = double(v[cc]);
    } else if (task < NU + NUN4) {
      if (!a.dRdUn) continue;
      const int tk = task - NU;
      const int r = tk / (3 * D::NE), fk = tk % (3 * D::NE);
      jac_un4<D, R>(s.tab, s.p, r, fk / D::NE, fk % D::NE, v);
      double* o = a.dRdUn + ((long long)e * D::NUE + r) * D::NUN + 4 * fk;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) o[cc] = double(v[cc]);
    } else {
      if (!a.dRdx) continue;
      const int tk = task - NU - NUN4;
      const int r = tk / D::NN, kn = tk % D::NN;
      jac_x2<D, R>(s.tab, s.p, r, kn, v);
      double* o = a.dRdx + ((long long)e * D::NUE + r) * D::NXE + 2 * kn;
      o[0] = double(v[0]);
      o[1] = double(v[1]);
    }
  }
  if (tid == 0) {
    if (a.N) a.N[e] = double(s.p.N);
    a.flags[e] = s.p.bad;
  }
  if (a.dNdx && tid < D::NXE) a.dNdx[(long long)e * D::NXE + tid] = double(s.p.dN[tid]);
}

// Full-order element with all Jacobian blocks in one block (four state
// components): the point physics of k_points_hdm, then the outputs written
// from the same LDS, with no point-data round trip through memory.
template <class D, class R>
__global__ __launch_bounds__(NTHR_PTS) void k_hdm_fused(HdmArgs a) {
  __shared__ ElemLDS<D, R> s;
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  load_tab<D, R, NTHR_PTS>(s, tid);
  load_hdm<D, R>(s, a, e, tid, NTHR_PTS);
  __syncthreads();
  phase_points<D, R, true>(s, tid, a.pc, R(a.kappa), R(a.eps));
  __syncthreads();
  phase_distortion<D, R>(s, tid, R(a.kappa));
  __syncthreads();
  if constexpr (D::NC == 4) hdm_write_blocks<D, R>(s, a, e, tid, NTHR_PTS);
}

// The same for elements 2b and 2b+1 in one 256-thread block (four-component
// P2, phase_points_pair).  With an odd element count the last block computes
// its one element twice and writes it once.
template <class D, class R>
__global__ __launch_bounds__(2 * NTHR_PTS) void k_hdm_fused2(HdmArgs a) {
  __shared__ ElemLDS<D, R> s[2];
  const int e0 = 2 * blockIdx.x;
  const int tid = threadIdx.x, h = tid / NTHR_PTS, t = tid % NTHR_PTS;
  const int e = e0 + min(h, a.n_elem - 1 - e0);
  load_tab<D, R, NTHR_PTS>(s[h], t);
  load_hdm<D, R>(s[h], a, e, t, NTHR_PTS);
  __syncthreads();
  phase_points_pair<D, R>(s, tid, [&](int) -> const PhysConst& { return a.pc; }, R(a.eps));
  __syncthreads();
  phase_distortion<D, R>(s[h], t, R(a.kappa));
  __syncthreads();
  if (e == e0 + h) hdm_write_blocks<D, R>(s[h], a, e, t, NTHR_PTS);
}

template <class D, class R>
__global__ __launch_bounds__(NTHR_PTS) void k_points_hdm(HdmArgs a) {
  __shared__ ElemLDS<D, R> s;
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  load_tab<D, R, NTHR_PTS>(s, tid);
  load_hdm<D, R>(s, a, e, tid, NTHR_PTS);
  __syncthreads();
  static_assert(n_point_tasks<D, true>() <= NTHR_PTS, "one task per thread");
  phase_points<D, R, true>(s, tid, a.pc, R(a.kappa), R(a.eps));
  __syncthreads();
  phase_distortion<D, R>(s, tid, R(a.kappa));
  __syncthreads();
  copy_pts<D, R, NTHR_PTS>(reinterpret_cast<Pts<D, R>*>(a.pts) + e, &s.p, tid);
}

// Point data of sampled element k at evaluation point pt (one block).
// After the point physics and its barrier, for the EQ point kernels (one
// element of NTHR_PTS threads, two waves): the distortion terms
// (phase_distortion, first wave) and the distortion row of the projection,
// dv_j = sum_c dN_c Psi_e[c][j] for j < m (second wave, whose column loads
// issue while the first wave forms dN).  Ends with a barrier.
template <class D, class R>
IFT_DEV void phase_distortion_eq(ElemLDS<D, R>& s, const EqArgs& a, int k, int t) {
  const int m = a.m, j = t - 64;
  const bool own = j >= 0 && j < m;
  double ps[D::NXE];
  if (own) {
    const double* col = a.LiftX + ((long long)k * m + j) * D::NXE;
#pragma unroll
    for (int c = 0; c < D::NXE; ++c) ps[c] = col[c];
  }
  phase_distortion<D, R>(s, t, R(a.kappa));
  __syncthreads();
  if (own) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < D::NXE; ++c) acc += double(s.p.dN[c]) * ps[c];
    s.p.dv[j] = R(acc);
  }
  __syncthreads();
}

// One element at point pt.  The point's physical constants: a.pcs[pt] (or
// a.pc) in the multi-point calls, formed from a.mu when FROM_MU (the batched
// kernel, whose items each carry their instance's mu).
template <class D, class R, bool FROM_MU = false>
IFT_DEV void points_eq_body(ElemLDS<D, R>& s, const EqArgs& a, int k, int pt, int tid) {
  load_tab<D, R, NTHR_PTS>(s, tid);
  load_eq<D, R>(s, a, k, pt, tid);
  __syncthreads();
  const PhysConst pc = FROM_MU ? (a.mu ? phys_from_mu(a.pc, D::PDE, a.bc_mu_scale, a.mu + 2 * pt) : a.pc)
                               : point_consts(a, pt);
  static_assert(n_point_tasks<D, true>() <= NTHR_PTS, "one task per thread");
  phase_points<D, R, true>(s, tid, pc, R(a.kappa), R(a.eps));
  __syncthreads();
  phase_distortion_eq<D, R>(s, a, k, tid);
  copy_pts<D, R, NTHR_PTS>(reinterpret_cast<Pts<D, R>*>(a.pts) + ((long long)pt * a.n_s + k), &s.p, tid);
}

template <class D, class R>
__global__ __launch_bounds__(NTHR_PTS) void k_points_eq(EqArgs a) {
  __shared__ ElemLDS<D, R> s;
  const int k = blockIdx.x, pt = blockIdx.y;
  if (k >= a.n_s) return;   // the element axis is padded to a multiple of 8 (one XCD per element)
  points_eq_body<D, R>(s, a, k, pt, threadIdx.x);
}

// Point data of sampled elements 2b and 2b+1 at evaluation point pt (one
// 256-thread block, phase_points_pair).  With an odd n_s the last block
// computes its one element twice and writes it once.
template <class D, class R>
__global__ __launch_bounds__(2 * NTHR_PTS) void k_points_eq2(EqArgs a) {
  __shared__ ElemLDS<D, R> s[2];
  const int k0 = 2 * blockIdx.x, pt = blockIdx.y;
  if (k0 >= a.n_s) return;   // padding blocks (whole block)
  const int tid = threadIdx.x, h = tid / NTHR_PTS, t = tid % NTHR_PTS;
  const int k = k0 + min(h, a.n_s - 1 - k0);
  // ends with a barrier; FP32 takes 16-column chunks (three waves per SIMD).  The
  // reference table is copied once the lift's first loads are in flight.
  load_eq<D, R, sizeof(R) == 8 ? 32 : 16>(s[h], a, k, pt, t, [&] { load_tab<D, R, NTHR_PTS>(s[h], t); });
  const PhysConst pc = point_consts(a, pt);
  phase_points_pair<D, R>(s, tid, [&](int) -> const PhysConst& { return pc; }, R(a.eps));
  __syncthreads();
  phase_distortion_eq<D, R>(s[h], a, k, t);
  if (k == k0 + h)
    copy_pts<D, R, NTHR_PTS>(reinterpret_cast<Pts<D, R>*>(a.pts) + ((long long)pt * a.n_s + k), &s[h].p, t);
}

// ------------------------------------------------ full-order assembly
template <class D, class R>
__global__ __launch_bounds__(NTHR) void k_hdm_asm(HdmArgs a) {
  __shared__ ElemLDSJx<D, R> s;
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  load_tab<D, R, NTHR>(s, tid);
  copy_pts<D, R, NTHR>(&s.p, reinterpret_cast<const Pts<D, R>*>(a.pts) + e, tid);
  __syncthreads();
  if constexpr (D::NC == 4) {
    hdm_write_blocks<D, R>(s, a, e, tid, NTHR);
    return;
  }
  phase_assemble<D, R, true>(s, tid);
  __syncthreads();
  if (a.R && tid < D::NUE) a.R[(long long)e * D::NUE + tid] = double(s.Re[tid]);
  if (tid == 0) {
    if (a.N) a.N[e] = double(s.p.N);
    a.flags[e] = s.p.bad;
  }
  if (a.dNdx && tid < D::NXE) a.dNdx[(long long)e * D::NXE + tid] = double(s.p.dN[tid]);
  if (a.dRdU) {
    double* o = a.dRdU + (long long)e * D::NUE * D::NUE;
    for (int i = tid; i < D::NUE * D::NUE; i += NTHR) o[i] = double(s.Jx[i / D::NUE][i % D::NUE]);
  }
  if (a.dRdUn) {
    double* o = a.dRdUn + (long long)e * D::NUE * D::NUN;
    for (int i = tid; i < D::NUE * D::NUN; i += NTHR) o[i] = double(s.Jx[i / D::NUN][D::NUE + i % D::NUN]);
  }
  if (a.dRdx) {
    double* o = a.dRdx + (long long)e * D::NUE * D::NXE;
    for (int i = tid; i < D::NUE * D::NXE; i += NTHR) o[i] = double(s.Jx[i / D::NXE][D::NUE + D::NUN + i % D::NXE]);
  }
}

// ------------------------------------------------------------- EQ kernels
// ------------------------------------------------------------------------
// Values only, RV_LANES lanes per element: the 16 point tasks of an element
// (volume points, face points, distortion) run on the lanes of one group,
// so a block of RV_THR threads evaluates RV_SLOTS elements at once.  Each
// element keeps only its lifted data, point values and residual in LDS.
constexpr int RV_LANES = 16;
constexpr int RV_THR = 256;
constexpr int RV_SLOTS = RV_THR / RV_LANES;

template <class D, class R>
struct PtsVal : PtsSrc<D, R> {
  R fv[D::NQV][D::NC][2];
  R gp[D::NQV][D::NN][2];
  R H[3][D::NQF][D::NC];
  R N;
  int bad;
};

template <class D, class R>
struct ElemVal {
  R U[D::NUE];
  R Un[D::NUN];
  R x[D::NXE];
  R X[D::NXE];
  int face[3];
  PtsVal<D, R> p;
  R Re[D::NUE];
  R eta_ref;   // distortion of the reference element
};

template <class D, class R>
struct ResShared {
  RefTab tab;
  ElemVal<D, R> e[RV_SLOTS];
};

template <class D, class R>
IFT_DEV void res_load_tab(ResShared<D, R>& sh, int tid) {
  copy_obj<RefTab, RV_THR>(&sh.tab, &c_tab[D::P - 1], tid);
}

// One element (k, pt) per lane group; `act` is false for the groups of a
// block beyond the last item (they still reach every barrier).  j is the
// lane within the group.  Writes Jpart, flags and, if requested, the Ft rows
// and PTR, as the one-block-per-element kernel does.
template <class D, class R>
IFT_DEV void res_group_body(ResShared<D, R>& sh, ElemVal<D, R>& e, const EqArgs& a, int k, int pt, bool act,
                            int j) {
  static_assert(n_point_tasks<D, false>() <= RV_LANES, "one point task per lane");
  const RefTab& tab = sh.tab;
  const int n = a.n, m = a.m;
  if (act) {
    if (j < 3) e.face[j] = a.face_s[k * 3 + j];
    if (j == 0) e.p.bad = 0;
    if (j == 1) e.eta_ref = R(a.eta_ref_s[k]);
    const double* w = a.w + (long long)pt * n;
    const double* tau = a.tau + (long long)pt * m;
    constexpr int RU = D::NUE + D::NUN;
    const double* Lu = a.LiftU + (long long)k * n * RU;
    const double* Lx = a.LiftX + (long long)k * m * D::NXE;
    const double* Xs = a.X_s + (long long)k * D::NXE;
    for (int t = j; t < RU + D::NXE; t += RV_LANES) {
      if (t < RU) {
        const double acc = lift_dot(Lu + t, RU, w, n, 0.0);
        if (t < D::NUE) e.U[t] = R(acc);
        else e.Un[t - D::NUE] = R(acc);
      } else {
        const int q = t - RU;
        const double acc = lift_dot(Lx + q, D::NXE, tau, m, Xs[q]);
        e.x[q] = R(acc);
        e.X[q] = R(Xs[q]);
      }
    }
  }
  __syncthreads();
  if (act) {
    const PhysConst pc = a.mu ? phys_from_mu(a.pc, D::PDE, a.bc_mu_scale, a.mu + 2 * pt) : a.pc;
    if (j < D::NQV) {
      vol_point<D, R, R>(tab, e, j, -1, pc, R(a.eps));
    } else if (j < D::NQV + 3 * D::NQF) {
      const int r = j - D::NQV;
      face_point<D, R, R>(tab, e, r / D::NQF, r % D::NQF, -1, pc);
    } else if (j == D::NQV + 3 * D::NQF) {
      const Tan<R> eta = eta_elem<D, R>(tab, e.x, e.X, R(a.eps), -1);
      e.p.N = R(a.kappa) * (eta.v - e.eta_ref);
    }
  }
  __syncthreads();
  if (act) {
    const double sq = a.srho[k];
    const long long po = (long long)pt * a.nrows;
    double ss = 0.0;
    for (int r = j; r < D::NUE; r += RV_LANES) {
      const R v = residual_entry_p<D, R>(e.p, tab, r);
      e.Re[r] = v;
      ss += double(v) * double(v);
      if (a.Ft) a.Ft[po + (long long)k * D::NUE + r] = sq * double(v);
    }
    // fixed-order tree over the group's lanes
#pragma unroll
    for (int o = RV_LANES / 2; o > 0; o >>= 1) ss += __shfl_xor(ss, o, RV_LANES);
    if (j == 0) {
      ss += double(e.p.N) * double(e.p.N);
      a.Jpart[(long long)pt * a.n_s + k] = 0.5 * a.rho[k] * ss;
      a.flags[(long long)pt * a.n_s + k] = e.p.bad;
      if (a.Ft) a.Ft[po + (long long)a.n_s * D::NUE + k] = sq * double(e.p.N);
    }
  }
  if (a.PTR) {
    __syncthreads();
    if (act) {
      for (int c = j; c < n; c += RV_LANES) {
        double acc = 0.0;
        for (int r = 0; r < D::NUE; ++r) acc += a.Phi_s[((long long)k * D::NUE + r) * n + c] * double(e.Re[r]);
        a.PTR[((long long)pt * a.n_s + k) * n + c] = a.rho[k] * acc;
      }
    }
  }
  __syncthreads();
}

// Items pt * n_s + k over all evaluation points, RV_SLOTS per block.
template <class D, class R>
__global__ __launch_bounds__(RV_THR) void k_eq_res16(EqArgs a, int n_pts) {
  __shared__ ResShared<D, R> sh;
  const int tid = threadIdx.x, g = tid / RV_LANES, j = tid % RV_LANES;
  res_load_tab<D, R>(sh, tid);
  __syncthreads();
  const long long total = (long long)n_pts * a.n_s;
  const long long item = (long long)blockIdx.x * RV_SLOTS + g;
  const bool act = item < total;
  const int pt = act ? int(item / a.n_s) : 0, k = act ? int(item % a.n_s) : 0;
  res_group_body<D, R>(sh, sh.e[g], a, k, pt, act, j);
}

// ------------------------------------------------------------------------
// Full-order residual norms at reduced solutions, the indicator of the
// greedy search, eq. (greedy0): for evaluation point pt, element e lifts
// U_e = P_e^T Phi w, U_e' = P_e'^T Phi w (face-trace rows of the full basis)
// and x_e = Q_e^T (X + Psi tau), evaluates R_e (values only, RV_LANES lanes
// per element as k_eq_res16) and adds |R_e|^2.  Block b writes the sum of
// its RV_SLOTS elements and the number of invalid ones; k_hdm_norm_final
// adds the blocks of each point in block order.
struct HdmRomArgs {
  const double* Phi;   // [N_u][n]
  const double* Psi;   // [N_x][m]
  const double* w;     // [pt][n]
  const double* tau;   // [pt][m]
  const double* mu;    // [pt][2]
  const int* gn;       // [Ne][nn]
  const int* face;     // [Ne][3]
  const int* Pn;       // [Ne][nun]
  const double* X;     // [N_x]
  PhysConst pc;
  double eps, bc_mu_scale;
  int n, m, n_elem, nblk;
  double* part;        // [pt][nblk]
  int* nbad;           // [pt][nblk]
};

template <class D, class R>
__global__ __launch_bounds__(RV_THR) void k_hdm_res_rom(HdmRomArgs a) {
  static_assert(n_point_tasks<D, false>() <= RV_LANES, "one point task per lane");
  __shared__ ResShared<D, R> sh;
  __shared__ double ssum[RV_SLOTS];
  __shared__ int sbad[RV_SLOTS];
  const int tid = threadIdx.x, g = tid / RV_LANES, j = tid % RV_LANES;
  res_load_tab<D, R>(sh, tid);
  const int pt = blockIdx.y;
  const int e = blockIdx.x * RV_SLOTS + g;
  const bool act = e < a.n_elem;
  ElemVal<D, R>& el = sh.e[g];
  const int n = a.n, m = a.m;
  const double* w = a.w + (long long)pt * n;
  const double* tau = a.tau + (long long)pt * m;
  if (act) {
    if (j < 3) el.face[j] = a.face[e * 3 + j];
    if (j == 0) el.p.bad = 0;
    for (int t = j; t < D::NUE + D::NUN + D::NXE; t += RV_LANES) {
      if (t < D::NUE + D::NUN) {
        const long long row = t < D::NUE ? (long long)e * D::NUE + t : (long long)a.Pn[(long long)e * D::NUN + t - D::NUE];
        const double acc = row >= 0 ? lift_dot(a.Phi + row * n, 1, w, n, 0.0) : 0.0;
        if (t < D::NUE) el.U[t] = R(acc);
        else el.Un[t - D::NUE] = R(acc);
      } else {
        const int r = t - D::NUE - D::NUN;
        const long long c = 2LL * a.gn[(long long)e * D::NN + r / 2] + (r & 1);
        const double acc = lift_dot(a.Psi + c * m, 1, tau, m, a.X[c]);
        el.x[r] = R(acc);
        el.X[r] = R(a.X[c]);
      }
    }
  }
  __syncthreads();
  if (act) {
    const PhysConst pc = phys_from_mu(a.pc, D::PDE, a.bc_mu_scale, a.mu + 2 * pt);
    if (j < D::NQV) {
      vol_point<D, R, R>(sh.tab, el, j, -1, pc, R(a.eps));
    } else if (j < D::NQV + 3 * D::NQF) {
      const int r = j - D::NQV;
      face_point<D, R, R>(sh.tab, el, r / D::NQF, r % D::NQF, -1, pc);
    }
  }
  __syncthreads();
  double ss = 0.0;
  if (act)
    for (int r = j; r < D::NUE; r += RV_LANES) {
      const double v = double(residual_entry_p<D, R>(el.p, sh.tab, r));
      ss += v * v;
    }
#pragma unroll
  for (int o = RV_LANES / 2; o > 0; o >>= 1) ss += __shfl_xor(ss, o, RV_LANES);
  if (j == 0) {
    ssum[g] = ss;
    sbad[g] = act && el.p.bad != 0 ? 1 : 0;
  }
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    int b = 0;
    for (int q = 0; q < RV_SLOTS; ++q) {
      t += ssum[q];
      b += sbad[q];
    }
    a.part[(long long)pt * a.nblk + blockIdx.x] = t;
    a.nbad[(long long)pt * a.nblk + blockIdx.x] = b;
  }
}

// |R|_2 of each point from the block sums (fixed order), +inf if any
// element is invalid; n_bad (may be null) receives the count.
__global__ __launch_bounds__(256) void k_hdm_norm_final(const double* part, const int* nbad, int nblk, double* norms,
                                                        int* n_bad) {
  __shared__ double sp[256];
  __shared__ int sb[256];
  const int pt = blockIdx.x, t = threadIdx.x;
  double v = 0.0;
  int b = 0;
  for (int i = t; i < nblk; i += 256) {
    v += part[(long long)pt * nblk + i];
    b += nbad[(long long)pt * nblk + i];
  }
  sp[t] = v;
  sb[t] = b;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (t < d) {
      sp[t] += sp[t + d];
      sb[t] += sb[t + d];
    }
    __syncthreads();
  }
  if (t == 0) {
    norms[pt] = sb[0] ? __builtin_inf() : sqrt(sp[0]);
    if (n_bad) n_bad[pt] = sb[0];
  }
}

// ------------------------------------------------------------------------
// EQ assembly in factorized form.  With the point Jacobians of phase B,
//   A_e = dR/dU_e Phi_e + dR/dU_e' Phi_e' = Aw * Bw,
//   B_e = dR/dx_e Psi_e                  = Ax * Bx,
// where the A factors hold quadrature-point quantities of the evaluation
//   Aw: T [(i,c),(q,c')]   = -w_q sum_d gp[q][i][d] df/du[q][c][d][c'],
//       S-[(i,c),(f,q,c')] =  wf_q L_q(k_f(i)) dH/du-[f][q][c][c']   (0 if i not on f),
//       S+[(i,c),(f,q,c')] =  wf_q L_q(k_f(i)) dH/du+[f][q][c][c'],
//   Ax: [(i,c),(q,ab)]     =  w_q f_c . d(cof(J) grad phi_i)/dJ_ab,
//       [(i,c),(f,q,d)]    =  wf_q L_q(k_f(i)) dH/dn~ . dn~/dt_d,
// and the B factors hold the reduced bases at the same points, which depend
// only on the ROM and are built once at ROM creation (k_point_bases):
//   Bw: Phi_e at the volume points, the traces of Phi_e and Phi_e' at the
//       face points;  Bx: dJ_ab/dtau at the volume points and dt/dtau at the
//       face points (cof(J) and n~ are linear in x_e).
// Both products run on FP64 matrix cores; each lane generates its A operand
// from the point data in LDS and reads its B operand from global memory.
template <class D>
struct EqOp {
  static constexpr int KV = D::NQV * D::NC;          // volume block of Aw
  static constexpr int KF = 3 * D::NQF * D::NC;      // one face block of Aw
  static constexpr int KW = KV + 2 * KF;
  static constexpr int KWP = (KW + 3) & ~3;          // padded to the MFMA k-step
  static constexpr int KXV = 4 * D::NQV;             // volume block of Ax
  static constexpr int KXF = 3 * D::NQF * 2;         // face block of Ax
  // Burgers: one more row per volume point, the derivative of the source
  // through the mapped position (x_q = sum_j x_j phi_j(xi_q))
  static constexpr int KXQ = D::PDE == PDE_BURGERS ? D::NQV : 0;
  static constexpr int KX = KXV + KXF + KXQ;
  static constexpr int KXP = (KX + 3) & ~3;
};

template <class D, class R>
struct EqAsmLDS {
  RefTab tab;
  Pts<D, R> p;
  R Re[D::NUE];
};

// Entries of Aw and Ax.  The *_vol / *_face forms take the quadrature
// point, face and component directly; aw_entry / ax_entry map a column to
// them.  They never select between loaded values: every load executes,
// selects are between constants, and a choice between two loaded values is
// the exact blend a s + b (1 - s) with s in {0, 1} (finite operands).  The
// compiler otherwise sinks such loads into divergent branches, and one such
// lowering was seen to leave the wrong arm in some lanes.
IFT_DEV double pick(double a, double b, bool first) {
  const double s = first ? 1.0 : 0.0;
  return a * s + b * (1.0 - s);
}

template <class D, class R>
IFT_DEV double aw_vol(const RefTab& t, const Pts<D, R>& p, int i, int c, int q, int cc) {
  return -t.wv[q] * (double(p.gp[q][i][0]) * double(p.Af[q][c][0][cc]) +
                     double(p.gp[q][i][1]) * double(p.Af[q][c][1][cc]));
}

// The same with the side fixed at compile time: one load, no blend.
template <bool PLUS, class D, class R>
IFT_DEV double aw_face_s(const RefTab& t, const Pts<D, R>& p, int i, int c, int f, int q, int cc) {
  return t.wl[i][f][q] * double(PLUS ? p.dHp[f][q][c][cc] : p.dHm[f][q][c][cc]);
}

template <class D, class R>
IFT_DEV double aw_face(const RefTab& t, const Pts<D, R>& p, int i, int c, bool plus, int f, int q, int cc) {
  const double hp = double(p.dHp[f][q][c][cc]);
  const double hm = double(p.dHm[f][q][c][cc]);
  return t.wl[i][f][q] * pick(hp, hm, plus);
}

template <class D, class R>
IFT_DEV double ax_vol(const RefTab& t, const Pts<D, R>& p, int i, int c, int q, int ab) {
  // d/dJ_ab of w_q f_c . (cof(J) grad phi_i), cof(J) = [[J11, -J10], [-J01, J00]]
  const double px = t.dphiv[q][i][0], py = t.dphiv[q][i][1];
  const double f0 = double(p.fv[q][c][0]), f1 = double(p.fv[q][c][1]);
  const double sgn = (ab == 0 || ab == 3) ? -1.0 : 1.0;
  double v = (sgn * t.wv[q]) * pick(f1, f0, ab < 2) * pick(px, py, (ab & 1) != 0);
  if constexpr (D::PDE == PDE_BURGERS)   // source term -w_q phi_i s d det J / dJ_ab
    v -= (t.wv[q] * t.phiv[q][i]) * double(p.src[q][1 + ab]);
  return v;
}

template <class D, class R>
IFT_DEV double ax_face(const RefTab& t, const Pts<D, R>& p, int i, int c, int f, int q, int d) {
  // d/dt_d of n~ = (t_y, -t_x)
  const double h0 = double(p.dHn[f][q][c][0]), h1 = double(p.dHn[f][q][c][1]);
  return t.wl[i][f][q] * pick(-h1, h0, d == 0);
}

// ax_vol and ax_tail for the four-component discretisations with the
// lane's choice of operand made on the index (one load each; the lane's ab,
// d and cf are fixed over a kernel): the same values, in the same order of
// operations, as the blends above.
template <class D, class R>
IFT_DEV double ax_vol_i(const RefTab& t, const Pts<D, R>& p, int i, int c, int q, int ab) {
  static_assert(D::PDE != PDE_BURGERS, "no source term");
  const double sgn = (ab == 0 || ab == 3) ? -1.0 : 1.0;
  const double f = double(p.fv[q][c][ab < 2 ? 1 : 0]);
  const double d = t.dphiv[q][i][(ab & 1) ? 0 : 1];
  return (sgn * t.wv[q]) * f * d;
}
template <class D, class R>
IFT_DEV double ax_tail_i(const RefTab& t, const Pts<D, R>& p, int i, int c, int cf) {
  using O = EqOp<D>;
  static_assert(O::KXQ == 0, "no source-position rows");
  const int cff = cf < O::KXF ? cf : O::KXF - 1;
  const int f = cff / (2 * D::NQF), q = (cff >> 1) % D::NQF, d = cff & 1;
  const double h = double(p.dHn[f][q][c][d == 0 ? 1 : 0]);
  return t.wl[i][f][q] * (d == 0 ? -h : h);
}

// Column cf of the rows after the volume block of Ax: the face rows
// (f, q, d) and, for Burgers, the source-position rows q.
template <class D, class R>
IFT_DEV double ax_tail(const RefTab& t, const Pts<D, R>& p, int i, int c, int cf) {
  using O = EqOp<D>;
  const int cff = cf < O::KXF ? cf : O::KXF - 1;
  const double vf = ax_face<D, R>(t, p, i, c, cff / (2 * D::NQF), (cff >> 1) % D::NQF, cff & 1);
  if constexpr (O::KXQ > 0) {
    // -w_q phi_i b det J s_q against the row d x_q / d tau
    const int q = cf >= O::KXF ? cf - O::KXF : 0;
    const double vq = -(t.wv[q] * t.phiv[q][i]) * double(p.src[q][5]);
    return pick(vf, vq, cf < O::KXF);
  } else {
    return vf;
  }
}

template <class D, class R>
IFT_DEV double aw_entry(const RefTab& t, const Pts<D, R>& p, int r, int col) {
  using O = EqOp<D>;
  constexpr int NC = D::NC;
  const int rr = r < D::NUE ? r : 0;
  const int i = rr / NC, c = rr % NC;
  const int cv = col < O::KV ? col : O::KV - 1;
  const double vv = aw_vol<D, R>(t, p, i, c, cv / NC, cv % NC);
  const int cfa = col - O::KV;
  const bool plus = cfa >= O::KF;
  int cf = plus ? cfa - O::KF : cfa;
  cf = cf < 0 ? 0 : (cf >= O::KF ? O::KF - 1 : cf);
  const double vf = aw_face<D, R>(t, p, i, c, plus, cf / (D::NQF * NC), (cf / NC) % D::NQF, cf % NC);
  const double sv = col < O::KV ? 1.0 : 0.0;
  return (vv * sv + vf * (1.0 - sv)) * ((r < D::NUE && col < O::KW) ? 1.0 : 0.0);
}

template <class D, class R>
IFT_DEV double ax_entry(const RefTab& t, const Pts<D, R>& p, int r, int col) {
  using O = EqOp<D>;
  constexpr int NC = D::NC;
  const int rr = r < D::NUE ? r : 0;
  const int i = rr / NC, c = rr % NC;
  const int cv = col < O::KXV ? col : O::KXV - 1;
  const double vv = ax_vol<D, R>(t, p, i, c, cv >> 2, cv & 3);
  int cf = col - O::KXV;
  cf = cf < 0 ? 0 : (cf >= O::KX - O::KXV ? O::KX - O::KXV - 1 : cf);
  const double vf = ax_tail<D, R>(t, p, i, c, cf);
  const double sv = col < O::KXV ? 1.0 : 0.0;
  return (vv * sv + vf * (1.0 - sv)) * ((r < D::NUE && col < O::KX) ? 1.0 : 0.0);
}

// Reduced bases at the quadrature points, per sampled element (ROM creation):
//   Bw [n_s][KWP][n + 1], Bx [n_s][KXP][m + 1]; padded rows and the last
//   column are zero, so a lane whose output column lies outside the block
//   loads that zero instead of branching around its load.
template <class D>
__global__ __launch_bounds__(256) void k_point_bases(const double* Phi_s, const double* Phin_s, const double* Psi_s,
                                                     int n, int m, double* Bw, double* Bx) {
  using O = EqOp<D>;
  constexpr int NC = D::NC;
  const RefTab& t = c_tab[D::P - 1];
  const int k = blockIdx.x;
  const double* Ph = Phi_s + (long long)k * D::NUE * n;
  const double* Pn = Phin_s + (long long)k * D::NUN * n;
  const double* Ps = Psi_s + (long long)k * D::NXE * m;
  const int lw = n + 1, lx = m + 1;
  for (int e = threadIdx.x; e < O::KWP * lw; e += 256) {
    const int row = e / lw, j = e % lw;
    double a = 0.0;
    if (j < n) {
      if (row < O::KV) {
        const int q = row / NC, cc = row % NC;
        for (int jn = 0; jn < D::NN; ++jn) a += t.phiv[q][jn] * Ph[(jn * NC + cc) * n + j];
      } else if (row < O::KW) {
        const bool plus = row >= O::KV + O::KF;
        const int cf = row - O::KV - (plus ? O::KF : 0);
        const int f = cf / (D::NQF * NC), q = (cf / NC) % D::NQF, cc = cf % NC;
        for (int kk = 0; kk < D::NE; ++kk)
          a += t.L[q][kk] * (plus ? Pn[((f * D::NE + kk) * NC + cc) * n + j] : Ph[(t.en[f][kk] * NC + cc) * n + j]);
      }
    }
    Bw[((long long)k * O::KWP + row) * lw + j] = a;
  }
  for (int e = threadIdx.x; e < O::KXP * lx; e += 256) {
    const int row = e / lx, j = e % lx;
    double a = 0.0;
    if (j < m) {
      if (row < O::KXV) {
        const int q = row >> 2, ab = row & 3, ca = ab >> 1, db = ab & 1;
        for (int kn = 0; kn < D::NN; ++kn) a += Ps[(2 * kn + ca) * m + j] * t.dphiv[q][kn][db];
      } else if (row < O::KXV + O::KXF) {
        const int cf = row - O::KXV;
        const int f = cf / (2 * D::NQF), q = (cf >> 1) % D::NQF, d = cf & 1;
        for (int kk = 0; kk < D::NE; ++kk) a += t.dL[q][kk] * Ps[(2 * t.en[f][kk] + d) * m + j];
      } else if (row < O::KX) {
        // first coordinate of the mapped volume point q
        const int q = row - O::KXV - O::KXF;
        for (int kn = 0; kn < D::NN; ++kn) a += t.phiv[q][kn] * Ps[(2 * kn) * m + j];
      }
    }
    Bx[((long long)k * O::KXP + row) * lx + j] = a;
  }
}

// C = A * B for one element on 16x16x4 FP64 matrix cores: A (nue x K) is
// generated per lane by `aop(r, k)`, B (K x ncol, row stride ncol + 1, last
// column zero) is read from global memory; output tiles are dealt to the
// four waves.  Lane layout: A[i][k] from lane i + 16k, B[k][j] from lane
// j + 16k, accumulator register v of lane l holds C[l/16 + 4v][l%16].  The
// k-loop is straight-line code: out-of-range rows are multiplied by zero
// and out-of-range columns load the zero column.
template <class D, class AOp, class Out>
IFT_DEV void mfma_elem(int K, const double* B, int ncol, int wave, int lane, AOp aop, Out out) {
  constexpr int MT = (D::NUE + 15) / 16;
  const int NT = (ncol + 15) / 16;
  const int ld = ncol + 1;
  for (int tt = wave; tt < MT * NT; tt += NTHR / 64) {
    const int mt = tt % MT, nt = tt / MT;
    const int row = 16 * mt + (lane & 15);
    const int col = 16 * nt + (lane & 15);
    const int kl = lane >> 4;
    const int rowc = row < D::NUE ? row : D::NUE - 1;
    const double rmask = row < D::NUE ? 1.0 : 0.0;
    const int colc = col < ncol ? col : ncol;
    dvec4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 4) {
      const double av = aop(rowc, k0 + kl) * rmask;
      const double bv = B[(k0 + kl) * ld + colc];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * mt + kl + 4 * v;
      const int j = 16 * nt + (lane & 15);
      if (r < D::NUE && j < ncol) out(r, j, acc[v]);
    }
  }
}

template <class D, class R>
__global__ __launch_bounds__(NTHR) void k_eq_asm(EqArgs a, const double* Bw, const double* Bx) {
  using O = EqOp<D>;
  __shared__ EqAsmLDS<D, R> s;
  const int n = a.n, m = a.m, Dd = a.D;
  const int k = blockIdx.x, pt = blockIdx.y;
  const int tid = threadIdx.x;
  {
    const int* src = reinterpret_cast<const int*>(&c_tab[D::P - 1]);
    int* dst = reinterpret_cast<int*>(&s.tab);
    for (int i = tid; i < (int)(sizeof(RefTab) / sizeof(int)); i += NTHR) dst[i] = src[i];
  }
  copy_pts<D, R, NTHR>(&s.p, reinterpret_cast<const Pts<D, R>*>(a.pts) + ((long long)pt * a.n_s + k), tid);
  __syncthreads();
  const double sq = a.srho[k];
  const long long nrow_e = (long long)a.n_s * D::NUE;
  const long long po = (long long)pt * a.nrows;
  double* Jt = a.Jt + po * Dd;
  double* rows = Jt + (long long)k * D::NUE * Dd;
  const int wave = tid >> 6, lane = tid & 63;
  mfma_elem<D>(O::KWP, Bw + (long long)k * O::KWP * (n + 1), n, wave, lane,
               [&](int r, int c) { return aw_entry<D, R>(s.tab, s.p, r, c); },
               [&](int r, int j, double v) { rows[r * Dd + j] = sq * v; });
  if (m > 0)
    mfma_elem<D>(O::KXP, Bx + (long long)k * O::KXP * (m + 1), m, wave ^ 3, lane,
                 [&](int r, int c) { return ax_entry<D, R>(s.tab, s.p, r, c); },
                 [&](int r, int j, double v) { rows[r * Dd + n + j] = sq * v; });
  // distortion row sqrt(rho) [0, dN/dx_e Psi_e]
  const double* Ps = a.Psi_s + (long long)k * D::NXE * m;
  for (int j = tid; j < Dd; j += NTHR) {
    double acc = 0.0;
    if (j >= n)
      for (int c = 0; c < D::NXE; ++c) acc += double(s.p.dN[c]) * Ps[c * m + (j - n)];
    Jt[(nrow_e + k) * Dd + j] = sq * acc;
  }
  if (tid < D::NUE) {
    const R rv = residual_entry_p<D, R>(s.p, s.tab, tid);
    s.Re[tid] = rv;
    a.Ft[po + (long long)k * D::NUE + tid] = sq * double(rv);
  }
  __syncthreads();
  if (tid == 0) {
    double r2 = 0.0;
    for (int r = 0; r < D::NUE; ++r) r2 += double(s.Re[r]) * double(s.Re[r]);
    r2 += double(s.p.N) * double(s.p.N);
    a.Jpart[(long long)pt * a.n_s + k] = 0.5 * a.rho[k] * r2;
    a.flags[(long long)pt * a.n_s + k] = s.p.bad;
    a.Ft[po + nrow_e + k] = sq * double(s.p.N);
  }
}

// ------------------------------------- fused assembly and Gram (A10-A12)
// With the augmented element block
//   M_e = sqrt(rho_e) [ A_e        B_e              R_e ]   (rows 0..nue-1)
//                     [ 0   dN_e/dx_e Psi_e         N_e ]   (row nue)
// of D + 1 columns, sum_e M_e^T M_e holds H = J~^T J~ (leading D x D block),
// g = J~^T F~ (column D) and 2 J~ (corner).  Each wave owns E consecutive
// sampled elements of one evaluation point: it forms M_e as MT x NT FP64
// MFMA tiles and adds M_e^T M_e to NT(NT+1)/2 register tiles with a second
// MFMA.  That works without moving data because an accumulator register v
// of a tile holds rows 4v..4v+3 in exactly the lane order the A and B
// operands of the next MFMA expect.  The four waves of a block are added in
// wave order through LDS and the block writes one partial; k_fused_final
// adds the partials in block order, so the result is deterministic.
constexpr int FUSED_MAXNT = 3;
constexpr int GF_ENT = 16, GF_GRP = 16;   // final reductions: entries x block groups per workgroup

struct FusedArgs {
  int E;              // sampled elements per wave
  int nblk;           // blocks per evaluation point
  double* part;       // [pt][nblk][NT(NT+1)/2][256]   (register-major tiles)
  int* part_bad;      // [pt][nblk][2]  (count, OR of the invalid flags)
  int rows;           // also store the rows of J~ and F~ (Jt, Ft)
  int pts2;           // stacked points (k_eq_fused_pts2): blocks per point pair
};

template <class D, class R>
struct alignas(16) FusedSlot {
  Pts<D, R> p;
};

// One wave copies one element's point data (16-byte words where the array
// stride allows).
template <class D, class R>
IFT_DEV void copy_pts_wave(Pts<D, R>* dst, const Pts<D, R>* src, int lane) {
  if constexpr (sizeof(Pts<D, R>) % 16 == 0) {
    constexpr int nw = sizeof(Pts<D, R>) / 16;
    const int4* s4 = reinterpret_cast<const int4*>(src);
    int4* d4 = reinterpret_cast<int4*>(dst);
    for (int i = lane; i < nw; i += 64) d4[i] = s4[i];
  } else if constexpr (sizeof(Pts<D, R>) % 8 == 0) {
    constexpr int nw = sizeof(Pts<D, R>) / 8;
    const int2* s2 = reinterpret_cast<const int2*>(src);
    int2* d2 = reinterpret_cast<int2*>(dst);
    for (int i = lane; i < nw; i += 64) d2[i] = s2[i];
  } else {
    constexpr int nw = sizeof(Pts<D, R>) / 4;
    const int* s1 = reinterpret_cast<const int*>(src);
    int* d1 = reinterpret_cast<int*>(dst);
    for (int i = lane; i < nw; i += 64) d1[i] = s1[i];
  }
}

// One element's point data held in the registers of a wave (word i of the
// array in lane i % 64), so that the next element's copy can be in flight
// while the current element is assembled.  Words are 8 bytes where the
// array size allows, else 4.
template <class D, class R>
struct PtsRegs {
  using W = typename std::conditional<sizeof(Pts<D, R>) % 8 == 0, double, float>::type;
  static constexpr int NW = sizeof(Pts<D, R>) / sizeof(W);
  static constexpr int PER = (NW + 63) / 64;
};

template <class D, class R, class W, int PER>
IFT_DEV void pts_regs_load(W (&r)[PER], const Pts<D, R>* src, int lane) {
  constexpr int NW = PtsRegs<D, R>::NW;
  static_assert(PER == PtsRegs<D, R>::PER, "one register array per element");
  const W* s = reinterpret_cast<const W*>(src);
#pragma unroll
  for (int i = 0; i < PER - 1; ++i) r[i] = s[lane + 64 * i];
  const int j = lane + 64 * (PER - 1);
  r[PER - 1] = s[j < NW ? j : NW - 1];
}

template <class D, class R, class W, int PER>
IFT_DEV void pts_regs_store(const W (&r)[PER], Pts<D, R>* dst, int lane) {
  constexpr int NW = PtsRegs<D, R>::NW;
  static_assert(PER == PtsRegs<D, R>::PER, "one register array per element");
  W* d = reinterpret_cast<W*>(dst);
#pragma unroll
  for (int i = 0; i < PER - 1; ++i) d[lane + 64 * i] = r[i];
  const int j = lane + 64 * (PER - 1);
  if (j < NW) d[j] = r[PER - 1];
}

// Orders the LDS accesses of one wave around a hand-over between its lanes
// (a wave's LDS instructions execute in order; this keeps the compiler from
// moving accesses across the hand-over).
IFT_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS of the fused kernel: the reference table, one point-data slot per
// wave (reused for the cross-wave reduction) and the flag counts.
// Elements a wave assembles side by side (their MFMA and A-operand chains
// interleave, which hides the FP64 latencies at two waves per SIMD): two for
// the four-component discretisations up to two column tiles, one otherwise
// (three tiles of two elements do not fit 256 registers).
template <class D, int NT>
constexpr int fused_np() {
  return D::NC == 4 && NT <= 2 ? 2 : 1;
}

// Workgroups per CU the fused kernels are compiled for: two waves per SIMD
// (a 256-VGPR budget) when elements are assembled in pairs; otherwise as
// many as the single-element body allows at its width.
template <class D, int NT>
constexpr int fused_blocks_per_cu() {
  return fused_np<D, NT>() == 2 ? 2 : (NT == 1 ? 3 : (NT == 3 ? 2 : 1));
}

template <class D, class R, int NT>
struct FusedShared {
  RefTab tab;
  union {
    FusedSlot<D, R> w[NTHR / 64][fused_np<D, NT>()];
    double red[NTHR / 64 - 1][256];
  } u;
  int sbad[NTHR / 64][2];
};

template <class D, class R, int NT>
IFT_DEV void fused_load_tab(FusedShared<D, R, NT>& sh, int tid) {
  copy_obj<RefTab, NTHR>(&sh.tab, &c_tab[D::P - 1], tid);
}

// NP sampled elements k0, k0 + 1, ... of one wave, side by side, in the
// four-component discretisations: M_e of each formed tile by tile on FP64
// MFMA (A operands generated per lane from the element's point data in the
// wave's LDS slot, B operands the point bases), scaled by sqrt(rho_e), with
// the residual column and the distortion row inserted, and M_e^T M_e added
// to the Gram tiles h.  The w steps (a quadrature point, or a (face, point)
// pair, per step; the lane's column component is kl), then the x steps
// (volume: entry ab = kl of J at point q; faces: column 4 ks' + kl of the
// (face, point, direction) block), one loop per kind of step.  Each step
// issues its MFMAs with the B values in bc and then reloads bc with the B
// values of the next step (across the loops too), so those loads overlap
// the A values of the next step; the elements' chains interleave.  Tiles
// without w (x) columns skip the MFMAs of w (x) steps; the loads are issued
// for every tile.
template <class D, class R, int NT, int NP>
IFT_DEV void fused_elems4(FusedShared<D, R, NT>& sh, const EqArgs& a, const double* Bw, const double* Bx,
                          const FusedArgs& f, int pt, int k0, dvec4 (&h)[NT * (NT + 1) / 2], int& nbad, int& bor) {
  static_assert(D::NC == 4, "four-component discretisations");
  using O = EqOp<D>;
  constexpr int NUE = D::NUE;
  constexpr int MT = (NUE + 1 + 15) / 16;           // row tiles (element rows + distortion row)
  constexpr int RD_MT = NUE / 16, RD_K = (NUE % 16) % 4, RD_V = (NUE % 16) / 4;  // distortion row
  static_assert(O::KW == O::KWP, "w steps are whole points");
  constexpr int KWS = O::KWP / 4, KXS = O::KXP / 4;
  const RefTab& tab = sh.tab;
  const int n = a.n, m = a.m, Dd = a.D;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int kl = lane >> 4, li = lane & 15;
  const long long nrow_e = (long long)a.n_s * NUE;
  const long long po = (long long)pt * a.nrows;
  const int KS = KWS + (m > 0 ? KXS : 0);
  // per-lane row constants; rows past nue are multiplied by zero
  int ri[MT], rc[MT];
  double rm[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int row = 16 * mt + li;
    rm[mt] = row < NUE ? 1.0 : 0.0;
    ri[mt] = (row < NUE ? row : 0) / D::NC;
    rc[mt] = (row < NUE ? row : 0) % D::NC;
  }
  int cw[NT], cx[NT];
  bool won[NT], xon[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int c = 16 * nt + li, jx = c - n;
    cw[nt] = c < n ? c : n;
    cx[nt] = (jx >= 0 && jx < m) ? jx : m;
    won[nt] = 16 * nt < n;
    xon[nt] = 16 * nt + 16 > n && 16 * nt < n + m;
  }
  const Pts<D, R>* P[NP];
  const double* bw[NP];
  const double* bx[NP];
  double sq[NP], rv[NP];
  dvec4 acc[NP][MT][NT];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const int k = k0 + i;
    P[i] = &sh.u.w[wave][i].p;
    bw[i] = Bw + (long long)k * O::KWP * (n + 1);
    bx[i] = Bx + (long long)k * O::KXP * (m + 1);
    sq[i] = a.srho[k];
    // residual entry of row `lane` (row nue: the distortion)
    rv[i] = 0.0;
    if (lane < NUE) rv[i] = double(residual_entry_p<D, R>(*P[i], tab, lane));
    else if (lane == NUE) rv[i] = double(P[i]->N);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[i][mt][nt] = dvec4{0.0, 0.0, 0.0, 0.0};
  }
  double bc[NP][NT];
  auto bload = [&](int st) {
    st = st < KS ? st : KS - 1;
    const bool xs = st >= KWS;
    const int r = 4 * (xs ? st - KWS : st) + kl;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const double* base = xs ? bx[i] + (long long)r * (m + 1) : bw[i] + (long long)r * (n + 1);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) bc[i][nt] = base[xs ? cx[nt] : cw[nt]];
    }
  };
  auto mfmas = [&](const double (*av)[MT], const bool* on) {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      if (on[nt]) {
#pragma unroll
        for (int i = 0; i < NP; ++i)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
            acc[i][mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][mt], bc[i][nt], acc[i][mt][nt], 0, 0, 0);
      }
    }
  };
  bload(0);
#pragma unroll 1
  for (int q = 0; q < D::NQV; ++q) {
    double av[NP][MT];
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) av[i][mt] = aw_vol<D, R>(tab, *P[i], ri[mt], rc[mt], q, kl) * rm[mt];
    mfmas(av, won);
    bload(q + 1);
  }
  // face steps: the minus side's, then the plus side's (the side a template
  // argument of each loop)
  auto wface = [&](auto plus, int pl) {
#pragma unroll 1
    for (int fq = 0; fq < 3 * D::NQF; ++fq) {
      double av[NP][MT];
#pragma unroll
      for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          av[i][mt] = aw_face_s<decltype(plus)::value, D, R>(tab, *P[i], ri[mt], rc[mt], fq / D::NQF, fq % D::NQF,
                                                             kl) * rm[mt];
      mfmas(av, won);
      bload(D::NQV + 3 * D::NQF * pl + fq + 1);
    }
  };
  wface(std::false_type(), 0);
  wface(std::true_type(), 1);
  if (m > 0) {
#pragma unroll 1
    for (int q = 0; q < D::NQV; ++q) {
      double av[NP][MT];
#pragma unroll
      for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) av[i][mt] = ax_vol_i<D, R>(tab, *P[i], ri[mt], rc[mt], q, kl) * rm[mt];
      mfmas(av, xon);
      bload(KWS + q + 1);
    }
#pragma unroll 1
    for (int ks = 0; ks < KXS - D::NQV; ++ks) {
      const int cf0 = 4 * ks + kl;
      const double cm = cf0 < O::KX - O::KXV ? 1.0 : 0.0;
      const int cf = cf0 < O::KX - O::KXV ? cf0 : 0;
      double av[NP][MT];
#pragma unroll
      for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) av[i][mt] = ax_tail_i<D, R>(tab, *P[i], ri[mt], rc[mt], cf) * (rm[mt] * cm);
      mfmas(av, xon);
      bload(KWS + D::NQV + ks + 1);
    }
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const int k = k0 + i;
    // scale by sqrt(rho_e); insert the residual column and the distortion row
    // (its entry for x-column j: dv_j of the point data)
    double dsrc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int jd = 16 * nt + li - n;
      dsrc[nt] = (jd >= 0 && jd < m) ? double(P[i]->dv[jd]) : 0.0;
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * mt + kl + 4 * v;   // < 32
        const double rsrc = __shfl(rv[i], row);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int c = 16 * nt + li, jd = c - n;
          double x = sq[i] * acc[i][mt][nt][v];
          if (c == Dd) x = sq[i] * rsrc;   // zero below the distortion row
          else if (mt == RD_MT && kl == RD_K && v == RD_V && jd >= 0 && jd < m) x = sq[i] * dsrc[nt];
          acc[i][mt][nt][v] = x;
        }
      }
    if (f.rows) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = 16 * mt + kl + 4 * v, c = 16 * nt + li;
            if (row > NUE || c > Dd) continue;
            const long long gr = row < NUE ? (long long)k * NUE + row : nrow_e + k;
            if (c < Dd) a.Jt[(po + gr) * Dd + c] = acc[i][mt][nt][v];
            else a.Ft[po + gr] = acc[i][mt][nt][v];
          }
    }
    // Gram: rows 4v..4v+3 of row tile mt are the k-block of one MFMA step
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (16 * mt + 4 * v > NUE) continue;
        int t = 0;
#pragma unroll
        for (int ta = 0; ta < NT; ++ta)
#pragma unroll
          for (int tb = ta; tb < NT; ++tb, ++t)
            h[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(acc[i][mt][ta][v], acc[i][mt][tb][v], h[t], 0, 0, 0);
      }
    const int bad = P[i]->bad;
    nbad += bad != 0;
    bor |= bad;
    if (f.rows && lane == 0) a.flags[(long long)pt * a.n_s + k] = bad;
  }
}

// The block partial of evaluation point pt: the waves' Gram tiles h added
// in wave order through LDS (the slots' space: callers have finished with
// the point data), and the invalid-flag count and OR of the waves.
template <class D, class R, int NT>
IFT_DEV void fused_write_partial(FusedShared<D, R, NT>& sh, const FusedArgs& f, const dvec4 (&h)[NT * (NT + 1) / 2],
                                 int nbad, int bor, int pt, int blk) {
  constexpr int NH = NT * (NT + 1) / 2;
  auto& u = sh.u;
  auto& sbad = sh.sbad;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  __syncthreads();
  if (lane == 0) {
    sbad[wave][0] = nbad;
    sbad[wave][1] = bor;
  }
  double* part = f.part + ((long long)pt * f.nblk + blk) * NH * 256;
#pragma unroll
  for (int t = 0; t < NH; ++t) {
    if (wave > 0)
#pragma unroll
      for (int v = 0; v < 4; ++v) u.red[wave - 1][v * 64 + lane] = h[t][v];
    __syncthreads();
    if (wave == 0)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double x = h[t][v];
#pragma unroll
        for (int w = 0; w < NTHR / 64 - 1; ++w) x += u.red[w][v * 64 + lane];
        part[t * 256 + v * 64 + lane] = x;
      }
    __syncthreads();
  }
  if (tid == 0) {
    int c = 0, o = 0;
    for (int w = 0; w < NTHR / 64; ++w) {
      c += sbad[w][0];
      o |= sbad[w][1];
    }
    f.part_bad[((long long)pt * f.nblk + blk) * 2] = c;
    f.part_bad[((long long)pt * f.nblk + blk) * 2 + 1] = o;
  }
}

// One block of the fused assembly: sampled elements [4E blk, 4E (blk + 1))
// at evaluation point pt; writes the block's partial.  The table must be
// loaded; the first barrier inside makes it visible.
template <class D, class R, int NT>
IFT_DEV void fused_body(FusedShared<D, R, NT>& sh, const EqArgs& a, const double* Bw, const double* Bx,
                        const FusedArgs& f, int blk, int pt) {
  using O = EqOp<D>;
  constexpr int NUE = D::NUE;
  constexpr int MT = (NUE + 1 + 15) / 16;           // row tiles (element rows + distortion row)
  constexpr int NH = NT * (NT + 1) / 2;             // upper tiles of the Gram
  constexpr int RD_MT = NUE / 16, RD_K = (NUE % 16) % 4, RD_V = (NUE % 16) / 4;  // distortion row
  const RefTab& tab = sh.tab;
  auto& u = sh.u;
  auto& sbad = sh.sbad;
  const int n = a.n, m = a.m, Dd = a.D;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int kl = lane >> 4, li = lane & 15;
  dvec4 h[NH];
#pragma unroll
  for (int t = 0; t < NH; ++t) h[t] = dvec4{0.0, 0.0, 0.0, 0.0};
  int nbad = 0, bor = 0;
  const long long nrow_e = (long long)a.n_s * NUE;
  const long long po = (long long)pt * a.nrows;
  const int kbeg = (blk * (NTHR / 64) + wave) * f.E;
  // each wave owns its slots: the point data of the next elements are loaded
  // into registers while the current ones are assembled, and only the wave
  // synchronises
  const Pts<D, R>* pbase = reinterpret_cast<const Pts<D, R>*>(a.pts) + (long long)pt * a.n_s;
  if constexpr (D::NC == 4) {
    // groups of NP elements: the point data of the next group are loaded
    // into registers while the current group is assembled
    constexpr int NP = fused_np<D, NT>();
    typename PtsRegs<D, R>::W pre[NP][PtsRegs<D, R>::PER];
#pragma unroll
    for (int i = 0; i < NP; ++i)
      if (i < f.E && kbeg + i < a.n_s) pts_regs_load<D, R>(pre[i], pbase + kbeg + i, lane);
    __syncthreads();   // the table is loaded
    for (int e = 0; e < f.E;) {
      const int k = kbeg + e;
      if (k >= a.n_s) break;
      const int np = (NP == 2 && e + 1 < f.E && k + 1 < a.n_s) ? 2 : 1;   // wave-uniform
      wave_sync();     // the slots' previous contents are consumed
#pragma unroll
      for (int i = 0; i < NP; ++i)
        if (i < np) pts_regs_store<D, R>(pre[i], &u.w[wave][i].p, lane);
      const int en = e + np;
#pragma unroll
      for (int i = 0; i < NP; ++i)
        if (en + i < f.E && kbeg + en + i < a.n_s) pts_regs_load<D, R>(pre[i], pbase + kbeg + en + i, lane);
      wave_sync();
      if constexpr (NP == 2) {
        if (np == 2) fused_elems4<D, R, NT, 2>(sh, a, Bw, Bx, f, pt, k, h, nbad, bor);
        else fused_elems4<D, R, NT, 1>(sh, a, Bw, Bx, f, pt, k, h, nbad, bor);
      } else {
        fused_elems4<D, R, NT, 1>(sh, a, Bw, Bx, f, pt, k, h, nbad, bor);
      }
      e = en;
    }
  } else {
    FusedSlot<D, R>& S = u.w[wave][0];
    typename PtsRegs<D, R>::W pre[PtsRegs<D, R>::PER];
    if (kbeg < a.n_s) pts_regs_load<D, R>(pre, pbase + kbeg, lane);
    __syncthreads();   // the table is loaded
    for (int e = 0; e < f.E; ++e) {
      const int k = kbeg + e;
      if (k >= a.n_s) break;
      wave_sync();     // the slot's previous contents are consumed
      pts_regs_store<D, R>(pre, &S.p, lane);
      if (e + 1 < f.E && k + 1 < a.n_s) pts_regs_load<D, R>(pre, pbase + k + 1, lane);
      wave_sync();
      const Pts<D, R>& p = S.p;
      const double sq = a.srho[k];
      // residual entry of row `lane` (row nue: the distortion), distortion
      // row entry of x-column `lane`
      double rv = 0.0;
      if (lane < NUE) rv = double(residual_entry_p<D, R>(p, tab, lane));
      else if (lane == NUE) rv = double(p.N);
      const double dv = lane < m ? double(p.dv[lane]) : 0.0;   // distortion row entry of x-column `lane`
      // M_e projection: columns [0, n) from Aw * Bw, [n, D) from Ax * Bx
      dvec4 acc[MT][NT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = dvec4{0.0, 0.0, 0.0, 0.0};
      // per-lane row constants; rows past nue are multiplied by zero
      int ri[MT], rc[MT];
      double rm[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int row = 16 * mt + li;
        rm[mt] = row < NUE ? 1.0 : 0.0;
        ri[mt] = (row < NUE ? row : 0) / D::NC;
        rc[mt] = (row < NUE ? row : 0) % D::NC;
      }
      const double* bw = Bw + (long long)k * O::KWP * (n + 1);
      // one k-step of the w columns: A values av[mt] for columns 4 ks + kl
      auto wstep = [&](int ks, const double* av) {
        double bv[NT];   // loaded for every tile (tiles without w columns read the zero column)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int c = 16 * nt + li;
          bv[nt] = bw[(4 * ks + kl) * (n + 1) + (c < n ? c : n)];
        }
        // every tile takes part (a tile without w columns adds zeros), so the
        // k-loop is one basic block and the loads of later steps can be hoisted
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
            acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mt], bv[nt], acc[mt][nt], 0, 0, 0);
      };
#pragma unroll 4
      for (int ks = 0; ks < O::KWP / 4; ++ks) {
        double av[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) av[mt] = aw_entry<D, R>(tab, p, 16 * mt + li, 4 * ks + kl);
        wstep(ks, av);
      }
      if (m > 0) {
        const double* bx = Bx + (long long)k * O::KXP * (m + 1);
        auto xstep = [&](int ks, const double* av) {
          double bv[NT];
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const int jx = 16 * nt + li - n;
            bv[nt] = bx[(4 * ks + kl) * (m + 1) + ((jx >= 0 && jx < m) ? jx : m)];
          }
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
              acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mt], bv[nt], acc[mt][nt], 0, 0, 0);
        };
        // volume k-steps: quadrature point q, entry ab = kl of J
#pragma unroll 1
        for (int q = 0; q < D::NQV; ++q) {
          double av[MT];
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            av[mt] = ax_vol<D, R>(tab, p, ri[mt], rc[mt], q, kl) * rm[mt];
          }
          xstep(q, av);
        }
        // face k-steps: column 4 ks' + kl of the (face, point, direction) block
#pragma unroll 1
        for (int ks = 0; ks < (O::KXP - O::KXV) / 4; ++ks) {
          const int cf0 = 4 * ks + kl;
          const double cm = cf0 < O::KX - O::KXV ? 1.0 : 0.0;
          const int cf = cf0 < O::KX - O::KXV ? cf0 : 0;
          double av[MT];
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
            av[mt] = ax_tail<D, R>(tab, p, ri[mt], rc[mt], cf) * (rm[mt] * cm);
          xstep(D::NQV + ks, av);
        }
      }
      // scale by sqrt(rho_e); insert the residual column and the distortion row
      double dsrc[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int jd = 16 * nt + li - n;
        dsrc[nt] = __shfl(dv, (jd >= 0 && jd < 64) ? jd : 0);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * mt + kl + 4 * v;   // < 32
          const double rsrc = __shfl(rv, row);
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const int c = 16 * nt + li, jd = c - n;
            double x = sq * acc[mt][nt][v];
            if (c == Dd) x = sq * rsrc;   // zero below the distortion row
            else if (mt == RD_MT && kl == RD_K && v == RD_V && jd >= 0 && jd < m) x = sq * dsrc[nt];
            acc[mt][nt][v] = x;
          }
        }
      if (f.rows) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = 16 * mt + kl + 4 * v, c = 16 * nt + li;
              if (row > NUE || c > Dd) continue;
              const long long gr = row < NUE ? (long long)k * NUE + row : nrow_e + k;
              if (c < Dd) a.Jt[(po + gr) * Dd + c] = acc[mt][nt][v];
              else a.Ft[po + gr] = acc[mt][nt][v];
            }
      }
      // Gram: rows 4v..4v+3 of row tile mt are the k-block of one MFMA step
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (16 * mt + 4 * v > NUE) continue;
          int t = 0;
#pragma unroll
          for (int ta = 0; ta < NT; ++ta)
#pragma unroll
            for (int tb = ta; tb < NT; ++tb, ++t)
              h[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(acc[mt][ta][v], acc[mt][tb][v], h[t], 0, 0, 0);
        }
      const int bad = p.bad;
      nbad += bad != 0;
      bor |= bad;
      if (f.rows && lane == 0) a.flags[(long long)pt * a.n_s + k] = bad;
    }
  }
  fused_write_partial<D, R, NT>(sh, f, h, nbad, bor, pt, blk);
}

// ------------------------------------ multi-point calls: stacked points
// The evaluation points of a call share each sampled element's point bases.
// For a multi-point FP64 call a wave takes each of its elements at two
// points p0 = 2 pp and p1 = 2 pp + 1 together: the two points' 2 nue
// residual rows fill the MFMA row tiles (three for Euler P2, where two
// elements at one point take four, their distortion rows padding a tile
// each), and the B operands serve both.  A point's distortion row enters its
// Gram as a k-block of its own after its residual rows.  The x k-blocks run
// beside the w k-blocks (below), but within a column tile they reach
// disjoint columns, so every entry of M_e sums its terms in the one-point
// kernel's order and each element's M_e and Gram term are the same; only
// the grouping of elements into waves and blocks differs.

// LDS of the stacked-point kernel: the fused kernel's, plus a ring per wave
// of PTS2_RING slots filled PTS2_RING - 1 iterations ahead by direct loads
// that hold no registers.  Iteration i of the kernel takes w step i and, for
// i < KXP / 4, x step i; its slot holds the B stripe of each (four rows of Bw
// and of Bx: 32 (n + 1) and 32 (m + 1) bytes), the x stripe right after the
// w stripe, so one wave-wide load fills it when n + m <= 30.
constexpr int PTS2_RING = 4;
constexpr int PTS2_SLOT = 128;   // doubles: 32 (n + m + 2) bytes <= 1 KB
template <class D, int NT>
struct FusedShared2 {
  FusedShared<D, double, NT> f;
  alignas(16) double ring[NTHR / 64][PTS2_RING][PTS2_SLOT];
};

template <class D, int NT>
constexpr bool fused_pts2_ok() {
  return D::NC == 4 && NT <= 2 && D::NUE % 4 == 0 && (2 * D::NUE) % 16 == 0 &&
         (2 * D::NUE) / 16 < 2 * ((D::NUE + 1 + 15) / 16);
}

// Where the B stripes of one sampled element start (byte addresses; rows
// 4 i .. 4 i + 3 of its Bw and Bx blocks are iteration i's), and the lane's
// part of an iteration's load: lanes below 2 (n + 1) take 16 bytes of the w
// stripe, the next 2 (m + 1) lanes 16 bytes of the x stripe.
struct Pts2Stripes {
  unsigned long long w, x;   // this lane's word of iteration 0
  int sw, sx;                // stripe bytes
  bool lx;                   // the lane loads from the x stripe
  int nw, nwx;               // lanes of the w stripe, of both
};
template <class D>
IFT_DEV Pts2Stripes pts2_stripes(const double* Bw, const double* Bx, int n, int m, int k, int lane) {
  using O = EqOp<D>;
  Pts2Stripes b;
  b.sw = 32 * (n + 1);
  b.sx = 32 * (m + 1);
  b.nw = 2 * (n + 1);
  b.nwx = b.nw + 2 * (m + 1);
  b.lx = lane >= b.nw;
  b.w = reinterpret_cast<unsigned long long>(Bw + (long long)k * O::KWP * (n + 1)) + 16ull * (unsigned)lane;
  b.x = reinterpret_cast<unsigned long long>(Bx + (long long)k * O::KXP * (m + 1)) +
        16ull * (unsigned)(b.lx ? lane - b.nw : 0);
  return b;
}
// Issues iteration it's stripes into its slot of the wave's ring (the x
// stripe only while there are x steps).  The per-lane choice of stripe is a
// mask blend of the two addresses.
template <class D>
IFT_DEV void pts2_bdma(const Pts2Stripes& b, double* ring, int it, int lane) {
  constexpr int KXS = EqOp<D>::KXP / 4;
  const bool hx = it < KXS;
  const unsigned long long mx = b.lx ? ~0ull : 0ull;
  const unsigned long long aw = b.w + (unsigned long long)(it * b.sw);
  const unsigned long long ax = b.x + (unsigned long long)(it * b.sx);
  dma16_at(reinterpret_cast<const void*>((aw & ~mx) | (ax & mx)), ring + PTS2_SLOT * (it & (PTS2_RING - 1)),
           lane < (hx ? b.nwx : b.nw));
}

// Which column tiles the w and x steps reach (bit nt: w tile nt, bit NT + nt:
// x tile nt), fixed at compile time so that the steps carry no branches: the
// exact set for two tiles with n > 16, else every tile (a tile past the
// block's columns multiplies the zero column of the padded B rows).
template <int NT>
constexpr int pts2_tiles_all() {
  return (1 << (2 * NT)) - 1;
}
constexpr int PTS2_TILES_N17 = 0b1011;   // NT = 2, 16 < n: w tiles 0 and 1, x tile 1
template <int NT>
__host__ __device__ inline int pts2_tiles(int n, int m) {
  return (NT == 2 && n > 16 && n + m < 32) ? PTS2_TILES_N17 : pts2_tiles_all<NT>();
}
template <int MT, int NT, int MASK>
IFT_DEV void mfma_tiles(dvec4 (&acc)[MT][NT], const double* av, const double* b) {
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    if ((MASK >> nt) & 1) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mt], b[nt], acc[mt][nt], 0, 0, 0);
    }
  }
}

// Element k at the points in the wave's slots 0 and 1 (the slot-1 data may
// repeat slot 0: a lone last point, whose h1 the caller drops).
template <class D, int NT, int TILES>
IFT_DEV void fused_elem_pts2(FusedShared<D, double, NT>& sh, double* ring, const EqArgs& a, const double* Bw,
                             const double* Bx, int k,
                             dvec4 (&h0)[NT * (NT + 1) / 2], dvec4 (&h1)[NT * (NT + 1) / 2], int (&nbad)[2],
                             int (&bor)[2]) {
  static_assert(fused_pts2_ok<D, NT>(), "stacked points");
  using O = EqOp<D>;
  using R = double;
  constexpr int NUE = D::NUE;
  constexpr int MT = 2 * NUE / 16;                 // row tiles of the two points' residual rows
  constexpr int KWS = O::KWP / 4, KXS = O::KXP / 4;
  const RefTab& tab = sh.tab;
  const int n = a.n, m = a.m, Dd = a.D;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int kl = lane >> 4, li = lane & 15;
  const Pts<D, R>* P0 = &sh.u.w[wave][0].p;
  const Pts<D, R>* P1 = &sh.u.w[wave][1].p;
  // per-lane row constants: row 16 mt + li is row lr of point p
  const Pts<D, R>* Pm[MT];
  int ri[MT], rc[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int row = 16 * mt + li, p = row / NUE, lr = row - p * NUE;
    Pm[mt] = p ? P1 : P0;
    ri[mt] = lr / D::NC;
    rc[mt] = lr % D::NC;
  }
  // the lane's B entry of each column tile within a step's stripe
  constexpr int WT = TILES & ((1 << NT) - 1), XT = TILES >> NT;
  int ow[NT], ox[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int c = 16 * nt + li, jx = c - n;
    ow[nt] = kl * (n + 1) + (c < n ? c : n);
    ox[nt] = kl * (m + 1) + ((jx >= 0 && jx < m) ? jx : m);
  }
  const double sq = a.srho[k];
  const Pts2Stripes bst = pts2_stripes<D>(Bw, Bx, n, m, k, lane);
  // residual entry of row `lane` of each point
  const double rv0 = lane < NUE ? double(residual_entry_p<D, R>(*P0, tab, lane)) : 0.0;
  const double rv1 = lane < NUE ? double(residual_entry_p<D, R>(*P1, tab, lane)) : 0.0;
  dvec4 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = dvec4{0.0, 0.0, 0.0, 0.0};
  // B values of iteration it from its ring slot, after the stripes of
  // iteration it + PTS2_RING - 1 are issued (the caller issued the first
  // ones) and those of iteration it have landed.  The reads are volatile so
  // that they issue with the step's A-operand reads instead of being sunk
  // next to the MFMAs that use them.
  double bc[NT], bcx[NT];
  auto bstep = [&](int it, auto hx) {
    static_assert(PTS2_RING == 4, "the waits below count three iterations ahead");
    if (it + 3 < KWS) {
      pts2_bdma<D>(bst, ring, it + 3, lane);
      vm_wait<3>();
    } else if (it + 2 < KWS) {
      vm_wait<2>();
    } else if (it + 1 < KWS) {
      vm_wait<1>();
    } else {
      vm_wait<0>();
    }
    using lds_vdouble = const volatile __attribute__((address_space(3))) double;
    lds_vdouble* rs = (lds_vdouble*)(ring + PTS2_SLOT * (it & (PTS2_RING - 1)));
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) bc[nt] = (WT >> nt) & 1 ? rs[ow[nt]] : 0.0;
    if constexpr (decltype(hx)::value) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) bcx[nt] = (XT >> nt) & 1 ? rs[4 * (n + 1) + ox[nt]] : 0.0;
    }
  };
  const std::true_type with_x, plus_side;
  const std::false_type w_only, minus_side;
  // Iteration i: w step i and, while i < KXS, x step i (the kernel serves
  // ROMs with m > 0).  Both kinds open with their NQV volume steps; the x
  // face steps then run beside the first w face steps.  Each column tile adds
  // its k-steps in this order.
  constexpr int XF = KXS - D::NQV;   // x face steps
  static_assert(XF >= 0 && XF <= 6 * D::NQF, "x face steps beside the w face steps");
#pragma unroll 1
  for (int q = 0; q < D::NQV; ++q) {
    bstep(q, with_x);
    double av[MT], ax[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) av[mt] = aw_vol<D, R>(tab, *Pm[mt], ri[mt], rc[mt], q, kl);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) ax[mt] = ax_vol_i<D, R>(tab, *Pm[mt], ri[mt], rc[mt], q, kl);
    mfma_tiles<MT, NT, WT>(acc, av, bc);
    mfma_tiles<MT, NT, XT>(acc, ax, bcx);
  }
  // face steps fs = (side, face, point): the minus side's 3 NQF, then the
  // plus side's; the side is a template argument of each loop
  constexpr int NFS = 3 * D::NQF;
  static_assert(XF <= NFS, "x face steps beside the minus-side w face steps");
  auto wface = [&](auto plus, int fq, double* av) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
      av[mt] = aw_face_s<decltype(plus)::value, D, R>(tab, *Pm[mt], ri[mt], rc[mt], fq / D::NQF, fq % D::NQF, kl);
  };
#pragma unroll 1
  for (int fs = 0; fs < XF; ++fs) {
    bstep(D::NQV + fs, with_x);
    double av[MT], ax[MT];
    wface(minus_side, fs, av);
    const int cf0 = 4 * fs + kl;
    const double cm = cf0 < O::KX - O::KXV ? 1.0 : 0.0;
    const int cf = cf0 < O::KX - O::KXV ? cf0 : 0;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) ax[mt] = ax_tail_i<D, R>(tab, *Pm[mt], ri[mt], rc[mt], cf) * cm;
    mfma_tiles<MT, NT, WT>(acc, av, bc);
    mfma_tiles<MT, NT, XT>(acc, ax, bcx);
  }
#pragma unroll 1
  for (int fs = XF; fs < NFS; ++fs) {
    bstep(D::NQV + fs, w_only);
    double av[MT];
    wface(minus_side, fs, av);
    mfma_tiles<MT, NT, WT>(acc, av, bc);
  }
#pragma unroll 1
  for (int fs = 0; fs < NFS; ++fs) {
    bstep(D::NQV + NFS + fs, w_only);
    double av[MT];
    wface(plus_side, fs, av);
    mfma_tiles<MT, NT, WT>(acc, av, bc);
  }
  // scale by sqrt(rho_e) and insert the residual column.  The row's point
  // picks between two shuffled registers (a select, not a blend: a
  // non-finite residual of one point must not reach the other's rows).
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * mt + kl + 4 * v, p = row / NUE, lr = row - p * NUE;
      const double r0 = __shfl(rv0, lr), r1 = __shfl(rv1, lr);
      const double rsrc = p ? r1 : r0;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int c = 16 * nt + li;
        double x = sq * acc[mt][nt][v];
        if (c == Dd) x = sq * rsrc;
        acc[mt][nt][v] = x;
      }
    }
  // Gram: the k-blocks of rows 4v..4v+3 of tile mt, each within one point,
  // then each point's distortion row [0, dN_e Psi_e, N_e] as a k-block
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int p = (16 * mt + 4 * v) / NUE;
      int t = 0;
#pragma unroll
      for (int ta = 0; ta < NT; ++ta)
#pragma unroll
        for (int tb = ta; tb < NT; ++tb, ++t) {
          if (p == 0) h0[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(acc[mt][ta][v], acc[mt][tb][v], h0[t], 0, 0, 0);
          else h1[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(acc[mt][ta][v], acc[mt][tb][v], h1[t], 0, 0, 0);
        }
    }
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const Pts<D, R>* Pp = p ? P1 : P0;
    const double Nv = double(Pp->N);
    double dk[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int c = 16 * nt + li, jd = c - n;
      const bool xd = kl == 0 && jd >= 0 && jd < m;
      const double dvv = double(Pp->dv[xd ? jd : 0]);
      // every load executes; the entry is the exact blend of the two
      const double sx = xd ? 1.0 : 0.0, sn = (kl == 0 && c == Dd) ? 1.0 : 0.0;
      dk[nt] = sq * (dvv * sx + Nv * sn);
    }
    int t = 0;
#pragma unroll
    for (int ta = 0; ta < NT; ++ta)
#pragma unroll
      for (int tb = ta; tb < NT; ++tb, ++t) {
        if (p == 0) h0[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(dk[ta], dk[tb], h0[t], 0, 0, 0);
        else h1[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(dk[ta], dk[tb], h1[t], 0, 0, 0);
      }
  }
  const int b0 = P0->bad, b1 = P1->bad;
  nbad[0] += b0 != 0;
  bor[0] |= b0;
  nbad[1] += b1 != 0;
  bor[1] |= b1;
}

// One block: its share of the sampled elements at points 2 pp and 2 pp + 1
// (a lone last point is taken twice and written once); writes the block's
// partial of each point.  The table must be loaded; the first
// barrier inside makes it visible.
template <class D, int NT, int TILES>
IFT_DEV void fused_pts2_body(FusedShared2<D, NT>& sh2, const EqArgs& a, const double* Bw, const double* Bx,
                             const FusedArgs& f, int blk, int pp, int n_pts) {
  constexpr int NH = NT * (NT + 1) / 2;
  constexpr int PB = (int)sizeof(Pts<D, double>);
  static_assert(PB % 16 == 0, "point data in 16-byte words");
  using O = EqOp<D>;
  static_assert(O::KWP / 4 >= PTS2_RING - 1, "the first stripes are w steps");
  FusedShared<D, double, NT>& sh = sh2.f;
  const int p0 = 2 * pp, p1 = min(2 * pp + 1, n_pts - 1);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double* ring = &sh2.ring[wave][0][0];
  dvec4 h0[NH], h1[NH];
#pragma unroll
  for (int t = 0; t < NH; ++t) h0[t] = h1[t] = dvec4{0.0, 0.0, 0.0, 0.0};
  int nbad[2] = {0, 0}, bor[2] = {0, 0};
  // Block blk takes the same elements at every point pair: the pair's n_s
  // elements split as evenly as the blocks allow, then as evenly over the
  // block's four waves.
  const int nb = gridDim.x;
  const int bcnt = a.n_s / nb + (blk < a.n_s % nb ? 1 : 0);
  const int bbeg = blk * (a.n_s / nb) + min(blk, a.n_s % nb);
  const int ecnt = bcnt / 4 + (wave < bcnt % 4 ? 1 : 0);
  const int kbeg = bbeg + wave * (bcnt / 4) + min(wave, bcnt % 4);
  const Pts<D, double>* pb0 = reinterpret_cast<const Pts<D, double>*>(a.pts) + (long long)p0 * a.n_s;
  const Pts<D, double>* pb1 = reinterpret_cast<const Pts<D, double>*>(a.pts) + (long long)p1 * a.n_s;
  __syncthreads();   // the table is loaded
  for (int e = 0; e < ecnt; ++e) {
    const int k = kbeg + e;
    wave_sync();     // the slots' and the ring's previous contents are consumed
    // the element's point data at both points straight into the wave's
    // slots, then the first B stripes; wait for all but those stripes
#pragma unroll
    for (int o = 0; o < PB; o += 1024) {
      dma16(reinterpret_cast<const char*>(pb0 + k) + o, reinterpret_cast<char*>(&sh.u.w[wave][0].p) + o, lane,
            (PB - o) / 16);
      dma16(reinterpret_cast<const char*>(pb1 + k) + o, reinterpret_cast<char*>(&sh.u.w[wave][1].p) + o, lane,
            (PB - o) / 16);
    }
    const Pts2Stripes bst = pts2_stripes<D>(Bw, Bx, a.n, a.m, k, lane);
#pragma unroll
    for (int it = 0; it < PTS2_RING - 1; ++it) pts2_bdma<D>(bst, ring, it, lane);
    vm_wait<PTS2_RING - 1>();
    wave_sync();
    fused_elem_pts2<D, NT, TILES>(sh, ring, a, Bw, Bx, k, h0, h1, nbad, bor);
  }
  fused_write_partial<D, double, NT>(sh, f, h0, nbad[0], bor[0], p0, blk);
  if (p1 != p0) fused_write_partial<D, double, NT>(sh, f, h1, nbad[1], bor[1], p1, blk);
}

template <class D, int NT, int TILES>
__global__ __launch_bounds__(NTHR, 2) void k_eq_fused_pts2(EqArgs a, const double* Bw, const double* Bx, FusedArgs f,
                                                            int n_pts) {
  __shared__ FusedShared2<D, NT> sh;
  fused_load_tab<D, double, NT>(sh.f, threadIdx.x);
  fused_pts2_body<D, NT, TILES>(sh, a, Bw, Bx, f, blockIdx.x, blockIdx.y, n_pts);
}

template <class D, class R, int NT>
__global__ __launch_bounds__(NTHR, (fused_blocks_per_cu<D, NT>())) void k_eq_fused(EqArgs a, const double* Bw, const double* Bx, FusedArgs f) {
  __shared__ FusedShared<D, R, NT> sh;
  fused_load_tab<D, R, NT>(sh, threadIdx.x);
  fused_body<D, R, NT>(sh, a, Bw, Bx, f, blockIdx.x, blockIdx.y);
}

// Sum of the block partials: workgroup x reduces 16 upper entries of the
// augmented Gram (H, g and the objective); its 16 thread groups take the
// blocks q, q + 16, ... and are then added in group order (fixed order).
// The extra last workgroup reduces the invalid flags.
// Count and OR of the invalid flags of nblk block partials (pairs in pb),
// by one whole wave: lane l takes blocks l, l + 64, ... and the lanes
// combine by shuffles (integers: the order does not matter).  Every lane
// ends with the totals.
IFT_DEV void flags_of_blocks(const int* pb, int nblk, int& c, int& o) {
  const int lane = threadIdx.x & 63;
  int cc = 0, oo = 0;
  for (int b = lane; b < nblk; b += 64) {
    cc += pb[2 * b];
    oo |= pb[2 * b + 1];
  }
#pragma unroll
  for (int sh = 32; sh > 0; sh >>= 1) {
    cc += __shfl_xor(cc, sh);
    oo |= __shfl_xor(oo, sh);
  }
  c = cc;
  o = oo;
}

IFT_DEV void fused_final_body(const double* part, const int* part_bad, int nblk, int NT, int D, double* H, double* g,
                              double* Jobj, int* n_bad, int* flag_or, int bx, int pt, double (*red)[GF_ENT]) {
  const int tid = threadIdx.x;
  const int NH = NT * (NT + 1) / 2;
  const int D1 = D + 1;
  const int nent = D1 * (D1 + 1) / 2;
  const int nbe = (nent + GF_ENT - 1) / GF_ENT;
  const int* pb = part_bad + (long long)pt * nblk * 2;
  if (bx == nbe) {
    if (tid < 64) {
      int c, o;
      flags_of_blocks(pb, nblk, c, o);
      if (tid == 0) {
        if (n_bad) n_bad[pt] = c;
        if (flag_or) flag_or[pt] = o;
      }
    }
    return;
  }
  // the workgroup of the objective entry (the last) needs the OR too; its
  // thread is in the first wave
  int obad = 0;
  if (bx == (nent - 1) / GF_ENT && tid < 64) {
    int c;
    flags_of_blocks(pb, nblk, c, obad);
  }
  const int el = tid % GF_ENT, q = tid / GF_ENT;
  const int e = bx * GF_ENT + el;
  // e -> (i, j), i <= j <= D, row-major over the upper triangle
  int i = 0, rem = e < nent ? e : 0;
  while (rem >= D1 - i) {
    rem -= D1 - i;
    ++i;
  }
  const int j = i + rem;
  const int ta = i / 16, tb = j / 16;
  const int t = ta * NT - ta * (ta - 1) / 2 + (tb - ta);
  const int r = i % 16, c = j % 16;
  const long long stride = (long long)NH * 256;
  const double* pp = part + (long long)pt * nblk * stride + t * 256 + (r / 4) * 64 + (r % 4) * 16 + c;
  double v = 0.0;
  if (e < nent)
    for (int b = q; b < nblk; b += GF_GRP) v += pp[b * stride];
  red[q][el] = v;
  __syncthreads();
  if (q != 0 || e >= nent) return;
  for (int w = 1; w < GF_GRP; ++w) v += red[w][el];
  if (j < D) {
    H[(long long)pt * D * D + (long long)i * D + j] = v;
    H[(long long)pt * D * D + (long long)j * D + i] = v;
  } else if (i < D) {
    g[(long long)pt * D + i] = v;
  } else {
    Jobj[pt] = obad ? __builtin_inf() : 0.5 * v;   // objective; +inf when any sampled element is invalid
  }
}

__global__ __launch_bounds__(256) void k_fused_final(const double* part, const int* part_bad, int nblk, int NT, int D,
                                                     double* H, double* g, double* Jobj, int* n_bad, int* flag_or) {
  __shared__ double red[GF_GRP][GF_ENT];
  fused_final_body(part, part_bad, nblk, NT, D, H, g, Jobj, n_bad, flag_or, blockIdx.x, blockIdx.y, red);
}

// ------------------------------------------------- Gram and objective
// H = J~^T J~ and g = J~^T F~ over the rows of one evaluation point.
// k_gram_part: block b owns the fixed row range [b*rows_per, ...), stages it
// in LDS, and its four row groups (64 threads each) accumulate 4x4 register
// tiles of H (and g) over interleaved rows; the groups are added in fixed
// order and the partial is stored entry-major (part[entry][block]).
// k_gram_final: one thread per entry adds the nblk contiguous partials in
// block order; an extra block adds the objective parts in element order.
constexpr int GRAM_MAXROWS = 128;

struct GramArgs {
  const double* Jt;      // [pt][nrows][D]
  const double* Ft;      // [pt][nrows]
  const double* Jpart;   // [pt][n_s]
  const int* flags;      // [pt][n_s]
  long long nrows;
  int n_s, D, nblk, rows_per;
  double* part;          // [pt][nblk][D*D + D]
  double* H;             // [pt][D][D]
  double* g;             // [pt][D]
  double* Jobj;          // [pt]
  int* n_bad;            // [pt] or null
  int* flag_or;          // [pt] or null
};

// Row groups per block: as many as fit beside the TD x TD tile threads.
IFT_DEV int gram_groups(int TD) { return TD * TD <= 64 ? 4 : (TD * TD <= 128 ? 2 : 1); }

__global__ __launch_bounds__(256) void k_gram_part(GramArgs a) {
  extern __shared__ double sh[];
  const int D = a.D;
  const int Dp = (D + 3) & ~3;                // padded row length
  const int TD = Dp / 4;                      // 4x4 tiles per dimension (<= 16)
  const int G = gram_groups(TD);
  const int gsz = 256 / G;
  const int pt = blockIdx.y;
  const int tid = threadIdx.x;
  const int grp = tid / gsz, lt = tid % gsz;  // row group, thread in group
  const int ld = Dp + 1;                      // row stride (last column: F~)
  double* rows = sh;                          // [rows_per][ld], reused for the group sums
  const double* Jt = a.Jt + (long long)pt * a.nrows * D;
  const double* Ft = a.Ft + (long long)pt * a.nrows;
  const long long r0 = (long long)blockIdx.x * a.rows_per;
  const int nr = (int)max(0LL, min((long long)a.rows_per, a.nrows - r0));
  for (int i = tid; i < nr * ld; i += 256) {
    const int r = i / ld, c = i % ld;
    rows[i] = c < D ? Jt[(r0 + r) * D + c] : (c == Dp ? Ft[r0 + r] : 0.0);
  }
  __syncthreads();
  const int ti = lt / TD, tj = lt % TD;       // this thread's 4x4 tile
  const bool act = lt < TD * TD;
  double acc[4][4], gacc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    gacc[i] = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  }
  if (act) {
    for (int r = grp; r < nr; r += G) {
      const double* row = rows + r * ld;
      double va[4], vb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        va[i] = row[4 * ti + i];
        vb[i] = row[4 * tj + i];
      }
      const double f = row[Dp];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        gacc[i] += va[i] * f;
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += va[i] * vb[j];
      }
    }
  }
  // groups 1..G-1 hand their sums to group 0 through LDS; group 0 adds them
  // in group order and stores the block's partial (entry-major)
  const int nred = TD * TD * 20;              // 16 H entries + 4 g entries per tile
  __syncthreads();
  if (grp > 0 && act) {
    double* mine = rows + (grp - 1) * nred + lt * 20;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int j = 0; j < 4; ++j) mine[i * 4 + j] = acc[i][j];
      mine[16 + i] = gacc[i];
    }
  }
  __syncthreads();
  if (grp == 0 && act) {
    for (int q = 1; q < G; ++q) {
      const double* o = rows + (q - 1) * nred + lt * 20;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += o[i * 4 + j];
        gacc[i] += o[16 + i];
      }
    }
    const int nent = D * D + D;
    double* pp = a.part + ((long long)pt * a.nblk + blockIdx.x) * nent;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 4 * ti + i;
      if (r >= D) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = 4 * tj + j;
        if (c < D) pp[r * D + c] = acc[i][j];
      }
      if (tj == 0) pp[D * D + r] = gacc[i];
    }
  }
}

// k_gram_final: block b (of ceil(nent/16)) reduces 16 consecutive entries;
// its 16 thread groups read the partials of 16 entries as 128-byte
// segments, group q taking blocks q, q+16, ...; the groups are then added
// in group order.  The extra last block reduces the objective.

__global__ __launch_bounds__(256) void k_gram_final(GramArgs a) {
  __shared__ double red[GF_GRP][GF_ENT];
  __shared__ double sj[256];
  __shared__ int sc[256], so[256];
  const int D = a.D;
  const int pt = blockIdx.y;
  const int tid = threadIdx.x;
  const int nent = D * D + D;
  const int nbe = (nent + GF_ENT - 1) / GF_ENT;
  if ((int)blockIdx.x < nbe) {
    const int el = tid % GF_ENT, q = tid / GF_ENT;
    const int e = blockIdx.x * GF_ENT + el;
    double v = 0.0;
    if (e < nent) {
      const double* pp = a.part + (long long)pt * a.nblk * nent + e;
      double v0 = 0.0, v1 = 0.0;
      int b = q;
      for (; b + GF_GRP < a.nblk; b += 2 * GF_GRP) {
        v0 += pp[(long long)b * nent];
        v1 += pp[(long long)(b + GF_GRP) * nent];
      }
      if (b < a.nblk) v0 += pp[(long long)b * nent];
      v = v0 + v1;
    }
    red[q][el] = v;
    __syncthreads();
    if (q == 0 && e < nent) {
      double s = 0.0;
      for (int g = 0; g < GF_GRP; ++g) s += red[g][el];
      if (e < D * D) a.H[(long long)pt * D * D + e] = s;
      else a.g[(long long)pt * D + (e - D * D)] = s;
    }
    return;
  }
  double v = 0.0;
  int c = 0, o = 0;
  for (int k = tid; k < a.n_s; k += 256) {
    v += a.Jpart[(long long)pt * a.n_s + k];
    const int f = a.flags[(long long)pt * a.n_s + k];
    c += f != 0;
    o |= f;
  }
  sj[tid] = v;
  sc[tid] = c;
  so[tid] = o;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
      sj[tid] += sj[tid + st];
      sc[tid] += sc[tid + st];
      so[tid] |= so[tid + st];
    }
    __syncthreads();
  }
  if (tid == 0) {
    a.Jobj[pt] = so[0] ? __builtin_inf() : sj[0];
    if (a.n_bad) a.n_bad[pt] = sc[0];
    if (a.flag_or) a.flag_or[pt] = so[0];
  }
}

// Objective sum (fixed order), invalid flags, n_bad (residual-only path and
// the full-order loop).
__global__ __launch_bounds__(256) void k_obj_final(const double* Jpart, const int* flags, int n, double* Jobj,
                                                   int* n_bad, int* flag_or) {
  __shared__ double sj[256];
  __shared__ int sc[256], so[256];
  const int pt = blockIdx.x;
  const int tid = threadIdx.x;
  double v = 0.0;
  int c = 0, o = 0;
  for (int k = tid; k < n; k += 256) {
    if (Jpart) v += Jpart[(long long)pt * n + k];
    int f = flags[(long long)pt * n + k];
    c += f != 0;
    o |= f;
  }
  sj[tid] = v;
  sc[tid] = c;
  so[tid] = o;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      sj[tid] += sj[tid + s];
      sc[tid] += sc[tid + s];
      so[tid] |= so[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (Jobj) Jobj[pt] = so[0] ? __builtin_inf() : sj[0];
    if (n_bad) n_bad[pt] = sc[0];
    if (flag_or) flag_or[pt] = so[0];
  }
}

__global__ void k_sum_rows(const double* part, int nrows, int ncols, double* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncols) return;
  double v = 0.0;
  for (int k = 0; k < nrows; ++k) v += part[(long long)k * ncols + j];
  out[j] = v;
}

// Column sums of Phi per solution component: out[c][j] = sum_i Phi[i*nc + c][j]
// (fixed order: per-thread strided sums, then a tree over the block).
__global__ __launch_bounds__(256) void k_phi_colsum(const double* Phi, long long n_nodes, int nc, int n, double* out) {
  __shared__ double red[256];
  const int c = blockIdx.x / n, j = blockIdx.x % n;
  double a = 0.0;
  for (long long i = threadIdx.x; i < n_nodes; i += 256) a += Phi[(i * nc + c) * n + j];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c * n + j] = red[0];
}

// ------------------------------------------------------------ gathers (A1)
__global__ void k_gather_rows(const double* src, int ncol, const long long* rows, long long nrows, double* dst) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows * ncol) return;
  const long long r = i / ncol;
  const int c = (int)(i - r * ncol);
  const long long sr = rows[r];
  dst[i] = sr >= 0 ? src[sr * ncol + c] : 0.0;
}

// Column-major copies of the gathered bases for the lift: column j of
// sampled element k holds Phi_e's rows then Phi_e''s rows (LU, [k][j][nue +
// nun]), and Psi_e's rows (LX, [k][j][nxe]).  One thread per entry.
__global__ void k_lift_bases(const double* Phi_s, const double* Phin_s, const double* Psi_s, int nue, int nun,
                             int nxe, int n, int m, long long n_s, double* LU, double* LX) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int ru = nue + nun;
  const long long nu = n_s * n * ru, nx = n_s * m * nxe;
  if (i < nu) {
    const long long k = i / ((long long)n * ru);
    const int rem = (int)(i - k * n * ru), j = rem / ru, r = rem % ru;
    LU[i] = r < nue ? Phi_s[(k * nue + r) * n + j] : Phin_s[(k * nun + r - nue) * n + j];
  } else if (i < nu + nx) {
    const long long ix = i - nu;
    const long long k = ix / ((long long)m * nxe);
    const int rem = (int)(ix - k * m * nxe), j = rem / nxe, r = rem % nxe;
    LX[ix] = Psi_s[(k * nxe + r) * m + j];
  }
}

// Distortion of each reference element (X_e in the mapping; only the mesh
// and the reference table enter), one thread per element.
template <class D>
__global__ __launch_bounds__(256) void k_eta_ref(const double* X, const int* gn, int n_elem, double* out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elem) return;
  double Xe[D::NXE];
#pragma unroll
  for (int r = 0; r < D::NXE; ++r) Xe[r] = X[2LL * gn[(long long)e * D::NN + r / 2] + (r & 1)];
  out[e] = eta_reference<D, double>(c_tab[D::P - 1], Xe);
}

// ------------------------------------------------- LM step (dense, FP64)
// (H + lambda diag(0_n, I_m)) dz = -g by Cholesky in one wave (D <= 64),
// over the leading ns unknowns (ns = D: the full step; ns = n: a step in w
// with tau fixed, dz_tau = 0); out = {failed (not SPD), |S~|, |T~|, g . dz}.
// L holds 64 x 64 doubles of LDS.
IFT_DEV void lm_solve_body(const double* H, const double* g, int D, int n, int ns, double lambda, double* dz,
                           double* out, double* L, double* y, int& fail) {
  const int t = threadIdx.x;
  for (int i = t; i < ns * ns; i += 64) {
    const int r = i / ns, c = i % ns;
    double v = H[r * D + c];
    if (r == c && r >= n) v += lambda;
    L[r * 64 + c] = v;
  }
  if (t == 0) fail = 0;
  __syncthreads();
  for (int j = 0; j < ns; ++j) {
    if (t == 0) {
      double s = L[j * 64 + j];
      for (int k = 0; k < j; ++k) s -= L[j * 64 + k] * L[j * 64 + k];
      if (!(s > 0.0)) fail = 1;
      L[j * 64 + j] = sqrt(s > 0.0 ? s : 1.0);
    }
    __syncthreads();
    for (int i = j + 1 + t; i < ns; i += 64) {
      double s = L[i * 64 + j];
      for (int k = 0; k < j; ++k) s -= L[i * 64 + k] * L[j * 64 + k];
      L[i * 64 + j] = s / L[j * 64 + j];
    }
    __syncthreads();
  }
  if (t == 0) {
    for (int i = 0; i < ns; ++i) {
      double s = -g[i];
      for (int k = 0; k < i; ++k) s -= L[i * 64 + k] * y[k];
      y[i] = s / L[i * 64 + i];
    }
    for (int i = ns - 1; i >= 0; --i) {
      double s = y[i];
      for (int k = i + 1; k < ns; ++k) s -= L[k * 64 + i] * y[k];
      y[i] = s / L[i * 64 + i];
    }
    double nS = 0.0, nT = 0.0, sl = 0.0;
    for (int i = 0; i < D; ++i) {
      const double yi = i < ns ? y[i] : 0.0;
      if (i < n) nS += g[i] * g[i];
      else nT += g[i] * g[i];
      sl += g[i] * yi;
      dz[i] = yi;
    }
    out[0] = fail;
    out[1] = sqrt(nS);
    out[2] = sqrt(nT);
    out[3] = sl;
  }
  __syncthreads();
}

__global__ __launch_bounds__(64) void k_lm_solve(const double* H, const double* g, int D, int n, int ns, double lambda,
                                                 double* dz, double* out) {
  __shared__ double L[64 * 64];
  __shared__ double y[64];
  __shared__ int fail;
  lm_solve_body(H, g, D, n, ns, lambda, dz, out, L, y, fail);
}

// ------------------------------------------ LM step by QR (TSQR, FP64)
// The least-squares form of the step, eq. (levmarq-step):
//   min | [J~_z; 0 sqrt(lambda) I] dz + [F~; 0] |,
// by Householder QR of the stacked rows [J~_z | -F~] (nrows rows) and, for
// lambda > 0, the m rows [0 .. sqrt(lambda) e_j .. | 0] of the mapping block.
// Only the leading ns unknowns are solved for (ns = D, or ns = n for a step
// in w with tau fixed and dz_tau = 0).
// Block b reduces rows [QR_RB b, QR_RB (b + 1)) (zero past the end) to the
// C x C triangle R_b (C = ns + 1: the unknowns and the right-hand side);
// the triangles are stacked and reduced again until one block remains, whose
// triangle [R_z c; 0 rho] gives R_z dz = c by back substitution.  Every sum
// runs in a fixed order.
constexpr int QR_RB = 128;     // rows per block (one per thread)
constexpr int QR_MAXC = 48;    // C = D + 1 <= QR_MAXC

struct QrArgs {
  const double* Jt;   // first level: J~_z [nrows][D] and F~ [nrows]
  const double* Ft;
  const double* src;  // later levels: stacked triangles [rows][C] (null on the first)
  int rows;           // rows of this level
  int nrows, D, n, ns, C;   // D: row length of J~_z, ns: unknowns solved for, C = ns + 1
  double sqlam;       // sqrt(lambda); the mapping rows exist when rows > nrows on the first level
  double* dst;        // [gridDim.x][C][C] triangles
  const double* g;    // last level: [D] gradient, for |S~|, |T~| and g . dz
  double* dz;         // last level: [D]
  double* out;        // last level: {failed, |S~|, |T~|, g . dz}
};

IFT_DEV double qr_wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__global__ __launch_bounds__(QR_RB) void k_qr_rows(QrArgs q, int last) {
  __shared__ double A[QR_MAXC][QR_RB];         // column-major: A[c][row]
  __shared__ double red[QR_RB / 64][QR_MAXC];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int C = q.C, D = q.D, ns = q.ns;
  const long long r = (long long)blockIdx.x * QR_RB + t;
  const bool in = r < q.rows;
  if (q.src) {
    for (int c = 0; c < C; ++c) A[c][t] = in ? q.src[r * C + c] : 0.0;
  } else if (in && r < q.nrows) {
    for (int c = 0; c < ns; ++c) A[c][t] = q.Jt[r * D + c];
    A[ns][t] = -q.Ft[r];
  } else {
    const int j = in ? int(r - q.nrows) : -1;   // mapping row j: sqrt(lambda) in column n + j
    for (int c = 0; c < C; ++c) A[c][t] = (j >= 0 && c == q.n + j) ? q.sqlam : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < C; ++j) {
    // column j below the diagonal: sigma = |A[j:, j]|^2
    const double x = A[j][t] * (t >= j ? 1.0 : 0.0);
    const double s = qr_wave_sum(x * x);
    if (lane == 0) red[wv][0] = s;
    __syncthreads();
    double sig = 0.0;
    for (int w = 0; w < QR_RB / 64; ++w) sig += red[w][0];
    const double ajj = A[j][j];
    __syncthreads();
    if (sig == 0.0) continue;   // already reduced (uniform)
    // H = I - beta v v^T with v = A[j:, j] - alpha e_j, alpha = -sign(a_jj) sqrt(sigma),
    // v^T v = 2 (sigma - a_jj alpha) > 0
    const double al = -copysign(sqrt(sig), ajj);
    const double beta = 1.0 / (sig - ajj * al);
    const double v = A[j][t] * (t > j ? 1.0 : 0.0) + (ajj - al) * (t == j ? 1.0 : 0.0);
    for (int c = j + 1; c < C; ++c) {
      const double d = qr_wave_sum(v * A[c][t]);
      if (lane == 0) red[wv][c] = d;
    }
    __syncthreads();
    for (int c = j + 1; c < C; ++c) {
      double d = 0.0;
      for (int w = 0; w < QR_RB / 64; ++w) d += red[w][c];
      A[c][t] -= beta * d * v;
    }
    if (t == j) A[j][j] = al;
    __syncthreads();
  }
  if (!last) {
    // row t of the block triangle: R[t][c] = A[c][t] for c >= t
    if (t < C) {
      double* o = q.dst + ((long long)blockIdx.x * C + t) * C;
      for (int c = 0; c < C; ++c) o[c] = A[c][t] * (c >= t ? 1.0 : 0.0);
    }
    return;
  }
  if (t == 0) {
    int fail = 0;
    for (int i = D - 1; i >= ns; --i) q.dz[i] = 0.0;
    for (int i = ns - 1; i >= 0; --i) {
      double v = A[ns][i];
      for (int k = i + 1; k < ns; ++k) v -= A[k][i] * q.dz[k];
      const double rii = A[i][i];
      if (!(fabs(rii) > 0.0)) fail = 1;
      q.dz[i] = fail ? 0.0 : v / rii;
    }
    double sS = 0.0, sT = 0.0, sl = 0.0;
    for (int i = 0; i < D; ++i) {
      const double gi = q.g[i];
      if (i < q.n) sS += gi * gi;
      else sT += gi * gi;
      sl += gi * q.dz[i];
    }
    q.out[0] = fail;
    q.out[1] = sqrt(sS);
    q.out[2] = sqrt(sT);
    q.out[3] = sl;
  }
}

// Elemental reduced residuals of eq. (ift-eqp-res0) from the stacked rows of
// one evaluation point, Jt = sqrt(rho) [A; a] and Ft = sqrt(rho) [R; N]:
// C[k][j] = (sum_r Jt[k nue + r][j] Ft[k nue + r] + Jt[n_s nue + k][j]
// Ft[n_s nue + k]) / rho_k, i.e. [S^(e_k); T^(e_k)] without the weight.
__global__ void k_elem_contrib(const double* Jt, const double* Ft, const double* rho, int n_s, int nue, int D,
                               double* C) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n_s * D) return;
  const int k = (int)(t / D), j = (int)(t % D);
  double v = 0.0;
  for (int r = 0; r < nue; ++r) {
    const long long row = (long long)k * nue + r;
    v += Jt[row * D + j] * Ft[row];
  }
  const long long rd = (long long)n_s * nue + k;
  v += Jt[rd * D + j] * Ft[rd];
  C[t] = v / rho[k];
}

__global__ void k_axpy2(const double* w, const double* tau, const double* dz, double alpha, int n, int m,
                        double* wo, double* to) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wo[i] = w[i] + alpha * dz[i];
  else if (i < n + m) to[i - n] = tau[i - n] + alpha * dz[i];
}

}  // namespace ift
