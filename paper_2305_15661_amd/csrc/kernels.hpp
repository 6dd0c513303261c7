// Kernels of the element loop (full order and EQ-sampled), the deterministic
// reductions, and the small dense solve of the Levenberg-Marquardt step.
//
// Values only (residual, objective): one fused kernel per element.
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
  PhysConst pc;
  double kappa, eps;
  int n_elem;
};

// EQ kernels: blockIdx.x = sampled element k, blockIdx.y = evaluation point.
// Per-point arrays are laid out point-major with the strides below.
struct EqArgs {
  int n_s, n, m, D;
  long long nrows;       // n_s*nue + n_s
  const int* eq_elem;    // [n_s]
  const int* face;       // [Ne][3]
  const double* rho;     // [n_s]
  const double* srho;    // [n_s] sqrt(rho)
  const double* Phi_s;   // [n_s][nue][n]
  const double* Phin_s;  // [n_s][nun][n]
  const double* Psi_s;   // [n_s][nxe][m]
  const double* X_s;     // [n_s][nxe]
  const double* w;       // [pt][n]
  const double* tau;     // [pt][m]
  const double* mu;      // [pt][2] on the device, or null: use pc
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
    pc.uinf[0] = 1.0 + bc_scale * mu[0];
  } else {
    const double M = mu[0], a = mu[1] * (M_PI / 180.0), c = sqrt(base.gamma);
    pc.uinf[0] = 1.0;
    pc.uinf[1] = M * c * cos(a);
    pc.uinf[2] = M * c * sin(a);
    pc.uinf[3] = 1.0 / (base.gamma - 1.0) + 0.5 * base.gamma * M * M;
  }
  return pc;
}

template <class D, class R>
IFT_DEV void copy_words(void* dst, const void* src, int tid, int nthr) {
  constexpr int nw = sizeof(Pts<D, R>) / sizeof(int);
  int* d = reinterpret_cast<int*>(dst);
  const int* s = reinterpret_cast<const int*>(src);
  for (int i = tid; i < nw; i += nthr) d[i] = s[i];
}

// ------------------------------------------------------------------ loaders
template <class D, class R>
IFT_DEV void load_hdm(ElemLDS<D, R>& s, const HdmArgs& a, int e, int tid, int nthr) {
  constexpr int ntask = D::NUE + D::NUN + 2 * D::NXE + 3;
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
      s.face[f] = a.face[e * 3 + f];
    }
  }
  if (tid == 0) s.p.bad = 0;
}

// Lift U_e = Phi_e w, U_e' = Phi_e' w, x_e = X_e + Psi_e tau straight from
// the gathered bases (rows are contiguous in global memory).
template <class D, class R>
IFT_DEV void load_eq(ElemLDS<D, R>& s, const EqArgs& a, int k, int pt, int tid, int nthr) {
  const int n = a.n, m = a.m;
  const double* w = a.w + (long long)pt * n;
  const double* tau = a.tau + (long long)pt * m;
  constexpr int ntask = D::NUE + D::NUN + D::NXE + 3;
  for (int t = tid; t < ntask; t += nthr) {
    if (t < D::NUE + D::NUN) {
      const double* row = t < D::NUE ? a.Phi_s + ((long long)k * D::NUE + t) * n
                                     : a.Phin_s + ((long long)k * D::NUN + (t - D::NUE)) * n;
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc += row[j] * w[j];
      if (t < D::NUE) s.U[t] = R(acc);
      else s.Un[t - D::NUE] = R(acc);
    } else if (t < D::NUE + D::NUN + D::NXE) {
      const int r = t - D::NUE - D::NUN;
      const double* row = a.Psi_s + ((long long)k * D::NXE + r) * m;
      const double X = a.X_s[(long long)k * D::NXE + r];
      double acc = X;
      for (int j = 0; j < m; ++j) acc += row[j] * tau[j];
      s.x[r] = R(acc);
      s.X[r] = R(X);
    } else {
      const int f = t - D::NUE - D::NUN - D::NXE;
      s.face[f] = a.face[a.eq_elem[k] * 3 + f];
    }
  }
  if (tid == 0) s.p.bad = 0;
}

// ------------------------------------------------- full order, values only
template <class D, class R>
__global__ __launch_bounds__(NTHR) void k_hdm_val(HdmArgs a) {
  __shared__ ElemLDS<D, R> s;
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  load_tab<D, R>(s, tid, NTHR);
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
template <class D, class R>
__global__ __launch_bounds__(NTHR_PTS) void k_points_hdm(HdmArgs a) {
  __shared__ ElemLDS<D, R> s;
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  load_tab<D, R>(s, tid, NTHR_PTS);
  load_hdm<D, R>(s, a, e, tid, NTHR_PTS);
  __syncthreads();
  static_assert(n_point_tasks<D, true>() <= NTHR_PTS, "one task per thread");
  phase_points<D, R, true>(s, tid, a.pc, R(a.kappa), R(a.eps));
  __syncthreads();
  copy_words<D, R>(reinterpret_cast<Pts<D, R>*>(a.pts) + e, &s.p, tid, NTHR_PTS);
}

template <class D, class R>
__global__ __launch_bounds__(NTHR_PTS) void k_points_eq(EqArgs a) {
  __shared__ ElemLDS<D, R> s;
  const int k = blockIdx.x, pt = blockIdx.y;
  const int tid = threadIdx.x;
  load_tab<D, R>(s, tid, NTHR_PTS);
  load_eq<D, R>(s, a, k, pt, tid, NTHR_PTS);
  __syncthreads();
  const PhysConst pc = a.mu ? phys_from_mu(a.pc, D::PDE, a.bc_mu_scale, a.mu + 2 * pt) : a.pc;
  static_assert(n_point_tasks<D, true>() <= NTHR_PTS, "one task per thread");
  phase_points<D, R, true>(s, tid, pc, R(a.kappa), R(a.eps));
  __syncthreads();
  copy_words<D, R>(reinterpret_cast<Pts<D, R>*>(a.pts) + ((long long)pt * a.n_s + k), &s.p, tid, NTHR_PTS);
}

// ------------------------------------------------ full-order assembly
template <class D, class R>
__global__ __launch_bounds__(NTHR) void k_hdm_asm(HdmArgs a) {
  __shared__ ElemLDS<D, R> s;
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  load_tab<D, R>(s, tid, NTHR);
  copy_words<D, R>(&s.p, reinterpret_cast<const Pts<D, R>*>(a.pts) + e, tid, NTHR);
  __syncthreads();
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
// Residual and objective parts at one evaluation point (values only).
template <class D, class R>
__global__ __launch_bounds__(NTHR) void k_eq_res(EqArgs a) {
  __shared__ ElemLDS<D, R> s;
  const int k = blockIdx.x, pt = blockIdx.y;
  const int tid = threadIdx.x;
  load_tab<D, R>(s, tid, NTHR);
  load_eq<D, R>(s, a, k, pt, tid, NTHR);
  __syncthreads();
  const PhysConst pc = a.mu ? phys_from_mu(a.pc, D::PDE, a.bc_mu_scale, a.mu + 2 * pt) : a.pc;
  phase_points<D, R, false>(s, tid, pc, R(a.kappa), R(a.eps));
  __syncthreads();
  phase_assemble<D, R, false>(s, tid);
  __syncthreads();
  const double sq = a.srho[k];
  const long long po = (long long)pt * a.nrows;
  if (a.Ft && tid < D::NUE) a.Ft[po + (long long)k * D::NUE + tid] = sq * double(s.Re[tid]);
  if (tid == 0) {
    double acc = 0.0;
    for (int r = 0; r < D::NUE; ++r) acc += double(s.Re[r]) * double(s.Re[r]);
    acc += double(s.p.N) * double(s.p.N);
    a.Jpart[(long long)pt * a.n_s + k] = 0.5 * a.rho[k] * acc;
    a.flags[(long long)pt * a.n_s + k] = s.p.bad;
    if (a.Ft) a.Ft[po + (long long)a.n_s * D::NUE + k] = sq * double(s.p.N);
  }
  if (a.PTR) {
    for (int j = tid; j < a.n; j += NTHR) {
      double acc = 0.0;
      for (int r = 0; r < D::NUE; ++r) acc += a.Phi_s[((long long)k * D::NUE + r) * a.n + j] * double(s.Re[r]);
      a.PTR[((long long)pt * a.n_s + k) * a.n + j] = a.rho[k] * acc;
    }
  }
}

// C[r][j] = sum_{k<K} Jx[r][a0 + k] B[k*ldb + j] for r < nue, j < ncol, on
// 16x16x4 FP64 matrix-core tiles; 16x16 output tiles are dealt to the waves
// round-robin.  Lane layout: A[i][k] from lane
// i + 16k, B[k][j] from lane j + 16k, accumulator register v of lane l
// holds C[l/16 + 4v][l%16].
template <class D, class R, class Out>
IFT_DEV void project_tiles(const ElemLDS<D, R>& s, int a0, int K, const double* B, int ldb, int ncol, int wave,
                           int lane, Out out) {
  constexpr int MT = (D::NUE + 15) / 16;
  const int NT = (ncol + 15) / 16;
  const int ntile = MT * NT;
  for (int t = wave; t < ntile; t += NTHR / 64) {
    const int mt = t % MT;   // row tile
    const int nt = t / MT;   // column tile
    const int row = 16 * mt + (lane & 15);
    const int col = 16 * nt + (lane & 15);
    const int kl = lane >> 4;
    dvec4 c = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int kk = k0 + kl;
      const double av = (row < D::NUE && kk < K) ? double(s.Jx[row][a0 + kk]) : 0.0;
      const double bv = (col < ncol && kk < K) ? B[kk * ldb + col] : 0.0;
      c = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, c, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * mt + kl + 4 * v;
      const int j = 16 * nt + (lane & 15);
      if (r < D::NUE && j < ncol) out(r, j, c[v]);
    }
  }
}

// Jacobian rows of the stacked least-squares problem at one evaluation point.
template <class D, class R>
__global__ __launch_bounds__(NTHR) void k_eq_asm(EqArgs a) {
  __shared__ ElemLDS<D, R> s;
  extern __shared__ double dyn[];
  const int n = a.n, m = a.m, Dd = a.D;
  double* V = dyn;                                  // [nue+nun][n]
  double* P = V + (D::NUE + D::NUN) * n;            // [nxe][m]
  const int k = blockIdx.x, pt = blockIdx.y;
  const int tid = threadIdx.x;
  load_tab<D, R>(s, tid, NTHR);
  copy_words<D, R>(&s.p, reinterpret_cast<const Pts<D, R>*>(a.pts) + ((long long)pt * a.n_s + k), tid, NTHR);
  {
    const double* src = a.Phi_s + (long long)k * D::NUE * n;
    for (int i = tid; i < D::NUE * n; i += NTHR) V[i] = src[i];
    src = a.Phin_s + (long long)k * D::NUN * n;
    for (int i = tid; i < D::NUN * n; i += NTHR) V[D::NUE * n + i] = src[i];
    src = a.Psi_s + (long long)k * D::NXE * m;
    for (int i = tid; i < D::NXE * m; i += NTHR) P[i] = src[i];
  }
  __syncthreads();
  phase_assemble<D, R, true>(s, tid);
  __syncthreads();
  const double sq = a.srho[k];
  const long long nrow_e = (long long)a.n_s * D::NUE;
  const long long po = (long long)pt * a.nrows;
  if (tid < D::NUE) a.Ft[po + (long long)k * D::NUE + tid] = sq * double(s.Re[tid]);
  if (tid == 0) {
    double acc = 0.0;
    for (int r = 0; r < D::NUE; ++r) acc += double(s.Re[r]) * double(s.Re[r]);
    acc += double(s.p.N) * double(s.p.N);
    a.Jpart[(long long)pt * a.n_s + k] = 0.5 * a.rho[k] * acc;
    a.flags[(long long)pt * a.n_s + k] = s.p.bad;
    a.Ft[po + nrow_e + k] = sq * double(s.p.N);
  }
  // distortion row sqrt(rho) [0, dN/dx_e Psi_e]
  double* Jt = a.Jt + po * Dd;
  for (int j = tid; j < Dd; j += NTHR) {
    double acc = 0.0;
    if (j >= n)
      for (int c = 0; c < D::NXE; ++c) acc += double(s.p.dN[c]) * P[c * m + (j - n)];
    Jt[(nrow_e + k) * Dd + j] = sq * acc;
  }
  // element rows sqrt(rho) [dR/dU_e Phi_e + dR/dU_e' Phi_e', dR/dx_e Psi_e]
  const int wave = tid >> 6, lane = tid & 63;
  double* rows = Jt + (long long)k * D::NUE * Dd;
  project_tiles<D, R>(s, 0, D::NUE + D::NUN, V, n, n, wave, lane,
                      [&](int r, int j, double v) { rows[r * Dd + j] = sq * v; });
  if (m > 0)
    project_tiles<D, R>(s, D::NUE + D::NUN, D::NXE, P, m, m, wave, lane,
                        [&](int r, int j, double v) { rows[r * Dd + n + j] = sq * v; });
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
IFT_DEV inline int gram_groups(int TD) { return TD * TD <= 64 ? 4 : (TD * TD <= 128 ? 2 : 1); }

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
constexpr int GF_ENT = 16, GF_GRP = 16;

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

// ------------------------------------------------------------ gathers (A1)
__global__ void k_gather_rows(const double* src, int ncol, const long long* rows, long long nrows, double* dst) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows * ncol) return;
  const long long r = i / ncol;
  const int c = (int)(i - r * ncol);
  const long long sr = rows[r];
  dst[i] = sr >= 0 ? src[sr * ncol + c] : 0.0;
}

// ------------------------------------------------- LM step (dense, FP64)
// Solves (H + lambda diag(0_n, I_m)) dz = -g by Cholesky on one wavefront;
// also returns |g_w|, |g_tau|, g.dz.  out: [0] status (0 ok, 1 not SPD),
// [1] |S~|, [2] |T~|, [3] slope.
__global__ __launch_bounds__(64) void k_lm_solve(const double* H, const double* g, int D, int n, double lambda,
                                                 double* dz, double* out) {
  __shared__ double L[64 * 64];
  __shared__ double y[64];
  __shared__ int fail;
  const int t = threadIdx.x;
  for (int i = t; i < D * D; i += 64) {
    const int r = i / D, c = i % D;
    double v = H[i];
    if (r == c && r >= n) v += lambda;
    L[r * 64 + c] = v;
  }
  if (t == 0) fail = 0;
  __syncthreads();
  for (int j = 0; j < D; ++j) {
    if (t == 0) {
      double s = L[j * 64 + j];
      for (int k = 0; k < j; ++k) s -= L[j * 64 + k] * L[j * 64 + k];
      if (!(s > 0.0)) fail = 1;
      L[j * 64 + j] = sqrt(s > 0.0 ? s : 1.0);
    }
    __syncthreads();
    for (int i = j + 1 + t; i < D; i += 64) {
      double s = L[i * 64 + j];
      for (int k = 0; k < j; ++k) s -= L[i * 64 + k] * L[j * 64 + k];
      L[i * 64 + j] = s / L[j * 64 + j];
    }
    __syncthreads();
  }
  if (t == 0) {
    for (int i = 0; i < D; ++i) {
      double s = -g[i];
      for (int k = 0; k < i; ++k) s -= L[i * 64 + k] * y[k];
      y[i] = s / L[i * 64 + i];
    }
    for (int i = D - 1; i >= 0; --i) {
      double s = y[i];
      for (int k = i + 1; k < D; ++k) s -= L[k * 64 + i] * y[k];
      y[i] = s / L[i * 64 + i];
    }
    double nS = 0.0, nT = 0.0, sl = 0.0;
    for (int i = 0; i < D; ++i) {
      if (i < n) nS += g[i] * g[i];
      else nT += g[i] * g[i];
      sl += g[i] * y[i];
      dz[i] = y[i];
    }
    out[0] = fail;
    out[1] = sqrt(nS);
    out[2] = sqrt(nT);
    out[3] = sl;
  }
}

__global__ void k_axpy2(const double* w, const double* tau, const double* dz, double alpha, int n, int m,
                        double* wo, double* to) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wo[i] = w[i] + alpha * dz[i];
  else if (i < n + m) to[i - n] = tau[i - n] + alpha * dz[i];
}

}  // namespace ift
