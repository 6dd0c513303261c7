// Kernels of the element loop (full order and EQ-sampled), the deterministic
// reductions, and the small dense solve of the Levenberg-Marquardt step.
#pragma once
#include "element.hpp"

namespace ift {

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
  PhysConst pc;
  double kappa, eps;
  int n_elem;
};

struct EqArgs {
  int n_s, n, m, D;
  const int* eq_elem;    // [n_s]
  const int* face;       // [Ne][3]
  const double* rho;     // [n_s]
  const double* srho;    // [n_s] sqrt(rho)
  const double* Phi_s;   // [n_s][nue][n]
  const double* Phin_s;  // [n_s][nun][n]
  const double* Psi_s;   // [n_s][nxe][m]
  const double* X_s;     // [n_s][nxe]
  const double* w;       // [n]
  const double* tau;     // [m]
  double* Jt;            // [n_s*nue + n_s][D]
  double* Ft;            // [n_s*nue + n_s]
  double* Jpart;         // [n_s]
  int* flags;            // [n_s]
  double* PTR;           // [n_s][n] or null
  PhysConst pc;
  double kappa, eps;
};

// ------------------------------------------------------------------ loaders
template <class D, class R>
IFT_DEV void load_hdm(ElemLDS<D, R>& s, const HdmArgs& a, int e, int lane) {
  constexpr int ntask = D::NUE + D::NUN + 2 * D::NXE + 3;
  for (int k = lane; k < ntask; k += 64) {
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
  if (lane == 0) s.bad = 0;
}

// Lift U_e = Phi_e w, U_e' = Phi_e' w, x_e = X_e + Psi_e tau.
template <class D, class R>
IFT_DEV void load_eq(ElemLDS<D, R>& s, const EqArgs& a, int k, int lane) {
  constexpr int ntask = D::NUE + D::NUN + D::NXE + 3;
  const int n = a.n, m = a.m;
  for (int t = lane; t < ntask; t += 64) {
    if (t < D::NUE) {
      const double* row = a.Phi_s + ((long long)k * D::NUE + t) * n;
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc += row[j] * a.w[j];
      s.U[t] = R(acc);
    } else if (t < D::NUE + D::NUN) {
      int r = t - D::NUE;
      const double* row = a.Phin_s + ((long long)k * D::NUN + r) * n;
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc += row[j] * a.w[j];
      s.Un[r] = R(acc);
    } else if (t < D::NUE + D::NUN + D::NXE) {
      int r = t - D::NUE - D::NUN;
      const double* row = a.Psi_s + ((long long)k * D::NXE + r) * m;
      double X = a.X_s[(long long)k * D::NXE + r];
      double acc = 0.0;
      for (int j = 0; j < m; ++j) acc += row[j] * a.tau[j];
      s.x[r] = R(X + acc);
      s.X[r] = R(X);
    } else {
      int f = t - D::NUE - D::NUN - D::NXE;
      s.face[f] = a.face[a.eq_elem[k] * 3 + f];
    }
  }
  if (lane == 0) s.bad = 0;
}

// --------------------------------------------------------------- hdm kernel
template <class D, class R, bool JAC>
__global__ __launch_bounds__(64) void k_hdm(HdmArgs a) {
  __shared__ ElemLDS<D, R> s;
  const int e = blockIdx.x;
  const int lane = threadIdx.x;
  load_hdm<D, R>(s, a, e, lane);
  __syncthreads();
  phase_points<D, R, JAC>(s, lane, a.pc, R(a.kappa), R(a.eps));
  __syncthreads();
  phase_residual<D, R>(s, lane);
  __syncthreads();
  if (a.R && lane < D::NUE) a.R[(long long)e * D::NUE + lane] = double(s.Re[lane]);
  if (lane == 0) {
    if (a.N) a.N[e] = double(s.N);
    a.flags[e] = s.bad;
  }
  if constexpr (JAC) {
    if (a.dNdx && lane < D::NXE) a.dNdx[(long long)e * D::NXE + lane] = double(s.dN[lane]);
    for (int j = lane; j < D::NDIR_HDM; j += 64) {
      R dR[D::NUE];
      if (j < D::NUE + D::NUN) {
        R dU[D::NUE], dUn[D::NUN];
#pragma unroll
        for (int r = 0; r < D::NUE; ++r) dU[r] = R(r == j ? 1 : 0);
#pragma unroll
        for (int r = 0; r < D::NUN; ++r) dUn[r] = R(r + D::NUE == j ? 1 : 0);
        column_state<D, R>(s, dU, dUn, dR);
        if (j < D::NUE) {
          if (a.dRdU)
            for (int r = 0; r < D::NUE; ++r) a.dRdU[((long long)e * D::NUE + r) * D::NUE + j] = double(dR[r]);
        } else if (a.dRdUn) {
          for (int r = 0; r < D::NUE; ++r)
            a.dRdUn[((long long)e * D::NUE + r) * D::NUN + (j - D::NUE)] = double(dR[r]);
        }
      } else {
        const int jj = j - D::NUE - D::NUN;
        R dx[D::NXE];
#pragma unroll
        for (int r = 0; r < D::NXE; ++r) dx[r] = R(r == jj ? 1 : 0);
        R dNv;
        column_map<D, R>(s, dx, dR, dNv);
        if (a.dRdx)
          for (int r = 0; r < D::NUE; ++r) a.dRdx[((long long)e * D::NUE + r) * D::NXE + jj] = double(dR[r]);
      }
    }
  }
}

// ----------------------------------------------------------- EQ residual
template <class D, class R>
__global__ __launch_bounds__(64) void k_eq_res(EqArgs a) {
  __shared__ ElemLDS<D, R> s;
  const int k = blockIdx.x;
  const int lane = threadIdx.x;
  load_eq<D, R>(s, a, k, lane);
  __syncthreads();
  phase_points<D, R, false>(s, lane, a.pc, R(a.kappa), R(a.eps));
  __syncthreads();
  phase_residual<D, R>(s, lane);
  __syncthreads();
  const double sq = a.srho[k];
  if (a.Ft && lane < D::NUE) a.Ft[(long long)k * D::NUE + lane] = sq * double(s.Re[lane]);
  if (lane == 0) {
    double acc = 0.0;
    for (int r = 0; r < D::NUE; ++r) acc += double(s.Re[r]) * double(s.Re[r]);
    acc += double(s.N) * double(s.N);
    a.Jpart[k] = 0.5 * a.rho[k] * acc;
    a.flags[k] = s.bad;
    if (a.Ft) a.Ft[(long long)a.n_s * D::NUE + k] = sq * double(s.N);
  }
  if (a.PTR) {
    for (int j = lane; j < a.n; j += 64) {
      double acc = 0.0;
      for (int r = 0; r < D::NUE; ++r) acc += a.Phi_s[((long long)k * D::NUE + r) * a.n + j] * double(s.Re[r]);
      a.PTR[(long long)k * a.n + j] = a.rho[k] * acc;
    }
  }
}

// ----------------------------------------------------------- EQ Jacobian
template <class D, class R>
__global__ __launch_bounds__(64) void k_eq_jac(EqArgs a) {
  __shared__ ElemLDS<D, R> s;
  const int k = blockIdx.x;
  const int lane = threadIdx.x;
  load_eq<D, R>(s, a, k, lane);
  __syncthreads();
  phase_points<D, R, true>(s, lane, a.pc, R(a.kappa), R(a.eps));
  __syncthreads();
  phase_residual<D, R>(s, lane);
  __syncthreads();
  const double sq = a.srho[k];
  const long long nrow_e = (long long)a.n_s * D::NUE;
  if (lane < D::NUE) a.Ft[(long long)k * D::NUE + lane] = sq * double(s.Re[lane]);
  if (lane == 0) {
    double acc = 0.0;
    for (int r = 0; r < D::NUE; ++r) acc += double(s.Re[r]) * double(s.Re[r]);
    acc += double(s.N) * double(s.N);
    a.Jpart[k] = 0.5 * a.rho[k] * acc;
    a.flags[k] = s.bad;
    a.Ft[nrow_e + k] = sq * double(s.N);
  }
  for (int j = lane; j < a.D; j += 64) {
    R dR[D::NUE];
    R dNv = R(0);
    if (j < a.n) {
      R dU[D::NUE], dUn[D::NUN];
#pragma unroll
      for (int r = 0; r < D::NUE; ++r) dU[r] = R(a.Phi_s[((long long)k * D::NUE + r) * a.n + j]);
#pragma unroll
      for (int r = 0; r < D::NUN; ++r) dUn[r] = R(a.Phin_s[((long long)k * D::NUN + r) * a.n + j]);
      column_state<D, R>(s, dU, dUn, dR);
    } else {
      const int jj = j - a.n;
      R dx[D::NXE];
#pragma unroll
      for (int r = 0; r < D::NXE; ++r) dx[r] = R(a.Psi_s[((long long)k * D::NXE + r) * a.m + jj]);
      column_map<D, R>(s, dx, dR, dNv);
    }
#pragma unroll
    for (int r = 0; r < D::NUE; ++r) a.Jt[((long long)k * D::NUE + r) * a.D + j] = sq * double(dR[r]);
    a.Jt[(nrow_e + k) * a.D + j] = sq * double(dNv);
  }
}

// ------------------------------------------------------ Gram (J~^T J~, J~^T F~)
// Stage 1: block c sums rows [c*rows_per, (c+1)*rows_per) into part[c][:],
// entries: the upper triangle (a <= b, row-major) then J~^T F~.
constexpr int GRAM_ROWS = 256;
constexpr int GRAM_TILE = 32;

__global__ __launch_bounds__(256) void k_gram_partial(const double* Jt, const double* Ft, long long nrows, int D,
                                                       double* part) {
  extern __shared__ double sh[];
  double* rows = sh;                       // [GRAM_TILE][D]
  double* fr = sh + GRAM_TILE * D;         // [GRAM_TILE]
  const int npair = D * (D + 1) / 2;
  const int nent = npair + D;
  const long long r0 = (long long)blockIdx.x * GRAM_ROWS;
  const long long r1 = min(nrows, r0 + GRAM_ROWS);
  double acc[12];
  int ia[12], ib[12];
  int cnt = 0;
  for (int p = threadIdx.x; p < nent && cnt < 12; p += blockDim.x, ++cnt) {
    if (p < npair) {
      // invert p -> (a, b) with a <= b in row-major upper-triangle order
      int a = 0, rem = p;
      while (rem >= D - a) { rem -= D - a; ++a; }
      ia[cnt] = a;
      ib[cnt] = a + rem;
    } else {
      ia[cnt] = p - npair;
      ib[cnt] = -1;
    }
    acc[cnt] = 0.0;
  }
  for (long long t0 = r0; t0 < r1; t0 += GRAM_TILE) {
    const int nt = (int)min((long long)GRAM_TILE, r1 - t0);
    __syncthreads();
    for (int i = threadIdx.x; i < nt * D; i += blockDim.x) rows[i] = Jt[t0 * D + i];
    for (int i = threadIdx.x; i < nt; i += blockDim.x) fr[i] = Ft[t0 + i];
    __syncthreads();
    for (int c = 0; c < cnt; ++c) {
      double v = acc[c];
      const int a = ia[c], b = ib[c];
      if (b >= 0) {
        for (int r = 0; r < nt; ++r) v += rows[r * D + a] * rows[r * D + b];
      } else {
        for (int r = 0; r < nt; ++r) v += rows[r * D + a] * fr[r];
      }
      acc[c] = v;
    }
  }
  for (int c = 0, p = threadIdx.x; c < cnt; ++c, p += blockDim.x) part[(long long)blockIdx.x * nent + p] = acc[c];
}

__global__ void k_gram_final(const double* part, int nblk, int D, double* H, double* g) {
  const int npair = D * (D + 1) / 2;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npair + D) return;
  double v = 0.0;
  for (int c = 0; c < nblk; ++c) v += part[(long long)c * (npair + D) + p];
  if (p < npair) {
    int a = 0, rem = p;
    while (rem >= D - a) { rem -= D - a; ++a; }
    const int b = a + rem;
    H[a * D + b] = v;
    H[b * D + a] = v;
  } else {
    g[p - npair] = v;
  }
}

// Objective sum (fixed order), invalid flags, n_bad.
__global__ __launch_bounds__(64) void k_obj_final(const double* Jpart, const int* flags, int n, double* Jobj,
                                                  int* n_bad, int* flag_or) {
  __shared__ double sj[64];
  __shared__ int sc[64], so[64];
  double v = 0.0;
  int c = 0, o = 0;
  for (int k = threadIdx.x; k < n; k += 64) {
    if (Jpart) v += Jpart[k];
    int f = flags[k];
    c += f != 0;
    o |= f;
  }
  sj[threadIdx.x] = v;
  sc[threadIdx.x] = c;
  so[threadIdx.x] = o;
  __syncthreads();
  for (int s = 32; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sj[threadIdx.x] += sj[threadIdx.x + s];
      sc[threadIdx.x] += sc[threadIdx.x + s];
      so[threadIdx.x] |= so[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (Jobj) *Jobj = so[0] ? __builtin_inf() : sj[0];
    if (n_bad) *n_bad = sc[0];
    if (flag_or) *flag_or = so[0];
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
