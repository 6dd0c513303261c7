// One DG element on one 64-lane wavefront.
//
// Discretisation (Section 2.3 of the paper, readings where it is silent):
//   R_e[i,c] = sum_faces int phi_i H_c(u-, u+, n~) ds - int grad_0 phi_i . F_c dX,
//   F = g f(U) G^{-T} (eq. (p2r-flux)).
// With J = dx/dxi and J0 = dX/dxi the volume integrand reduces to
// f(u) . (cof(J) grad_xi phi_i) per unit reference-triangle measure, where
// cof(J) = det(J) J^{-T} is linear in x_e in 2-D; the face term uses
// n~ = (t_y, -t_x), t = dx/ds along the edge (Nanson's relation).  The
// mapping validity test uses g = det J / det J0, and the distortion of
// eq. (dist_elem1) uses G = J J0^{-1}.
//
// Work split inside the wave (all data of one element staged in LDS):
//   A  load / lift the element DoFs U_e, U_e', x_e, X_e;
//   B  point physics: each lane evaluates one quadrature point, or one
//      (point, input direction) pair in tangent arithmetic, giving the point
//      fluxes and their exact Jacobians;
//   C  residual R_e: one lane per (node, component);
//   D  Jacobian columns: one lane per input direction (a reduced basis
//      vector, or a unit vector for the full-order blocks).
#pragma once
#include "physics.hpp"

namespace ift {

struct RefTab {
  double wv[6];          // volume weights (sum 1/2)
  double phiv[6][6];     // phi_node(xi_q)            [q][node]
  double dphiv[6][6][2]; // grad_xi phi_node(xi_q)    [q][node][dim]
  double wf[3];          // face weights on s in [0,1] (sum 1)
  double L[3][3];        // 1-D Lagrange on the edge  [q][k]
  double dL[3][3];       // its s-derivative          [q][k]
  int en[3][3];          // element node of edge node k of face f [f][k]
  int nfk[6][3];         // edge-node index of node i on face f, or -1
};

extern __constant__ RefTab c_tab[2];

template <int PDE_, int P_>
struct Disc {
  static constexpr int PDE = PDE_;
  static constexpr int P = P_;
  static constexpr int NC = NComp<PDE_>::value;
  static constexpr int NN = (P_ + 1) * (P_ + 2) / 2;
  static constexpr int NQV = P_ == 1 ? 3 : 6;
  static constexpr int NQF = P_ + 1;
  static constexpr int NUE = NN * NC;
  static constexpr int NUN = 3 * (P_ + 1) * NC;
  static constexpr int NXE = 2 * NN;
  static constexpr int NDIR_HDM = NUE + NUN + NXE;
};

enum { BAD_GEOM = 1, BAD_STATE = 2 };

template <class D, class R>
struct ElemLDS {
  R U[D::NUE];
  R Un[D::NUN];
  R x[D::NXE];
  R X[D::NXE];
  R fv[D::NQV][D::NC][2];
  R Af[D::NQV][D::NC][2][D::NC];
  R gp[D::NQV][D::NN][2];
  R H[3][D::NQF][D::NC];
  R dHm[3][D::NQF][D::NC][D::NC];
  R dHp[3][D::NQF][D::NC][D::NC];
  R dHn[3][D::NQF][D::NC][2];
  R Re[D::NUE];
  R N;
  R dN[D::NXE];
  int face[3];
  int bad;
};

// ----------------------------------------------------------------- phase B
template <class D, class T, class R>
IFT_DEV void jac2(const RefTab& t, int q, const T* x, T& J00, T& J01, T& J10, T& J11) {
  J00 = mk<T, R>(R(0)); J01 = J00; J10 = J00; J11 = J00;
#pragma unroll
  for (int k = 0; k < D::NN; ++k) {
    R a = R(t.dphiv[q][k][0]), b = R(t.dphiv[q][k][1]);
    J00 = J00 + x[2 * k] * a;
    J01 = J01 + x[2 * k] * b;
    J10 = J10 + x[2 * k + 1] * a;
    J11 = J11 + x[2 * k + 1] * b;
  }
}

// Distortion eta_e = sum_q w_q det J0 (|G|_F^2 / max(g, eps))^2 with
// G = J J0^{-1}, g = det J / det J0 (eq. (dist_elem1), 2/d = 1).
template <class D, class T, class R>
IFT_DEV T eta_elem(const RefTab& t, const T* x, const R* X, R eps) {
  T eta = mk<T, R>(R(0));
#pragma unroll
  for (int q = 0; q < D::NQV; ++q) {
    T J00, J01, J10, J11;
    jac2<D, T, R>(t, q, x, J00, J01, J10, J11);
    R K00, K01, K10, K11;
    jac2<D, R, R>(t, q, X, K00, K01, K10, K11);
    R dK = K00 * K11 - K01 * K10;
    R i00 = K11 / dK, i01 = -K01 / dK, i10 = -K10 / dK, i11 = K00 / dK;
    T G00 = J00 * i00 + J01 * i10, G01 = J00 * i01 + J01 * i11;
    T G10 = J10 * i00 + J11 * i10, G11 = J10 * i01 + J11 * i11;
    T nG2 = G00 * G00 + G01 * G01 + G10 * G10 + G11 * G11;
    T g = (J00 * J11 - J01 * J10) / dK;
    T mx = val(g) >= eps ? g : mk<T, R>(eps);
    T r = nG2 / mx;
    eta = eta + (R(t.wv[q]) * dK) * (r * r);
  }
  return eta;
}

// Volume point q: state, flux, cof(J) grad phi; seed = component seeded in
// tangent mode (-1: none).  Returns the flux Jacobian column in Af.
template <class D, class T, class R>
IFT_DEV void vol_point(ElemLDS<D, R>& s, const RefTab& t, int q, int seed, const PhysConst& pc, R eps) {
  T u[D::NC];
#pragma unroll
  for (int c = 0; c < D::NC; ++c) {
    R a = R(0);
#pragma unroll
    for (int j = 0; j < D::NN; ++j) a += R(t.phiv[q][j]) * s.U[j * D::NC + c];
    u[c] = seedv<T, R>(a, c == seed);
  }
  T f[D::NC][2];
  phys_flux<D::PDE, T, R>(u, f, R(pc.gamma));
  if (seed <= 0) {
#pragma unroll
    for (int c = 0; c < D::NC; ++c) {
      s.fv[q][c][0] = val(f[c][0]);
      s.fv[q][c][1] = val(f[c][1]);
    }
    R J00, J01, J10, J11, K00, K01, K10, K11;
    jac2<D, R, R>(t, q, s.x, J00, J01, J10, J11);
    jac2<D, R, R>(t, q, s.X, K00, K01, K10, K11);
    R g = (J00 * J11 - J01 * J10) / (K00 * K11 - K01 * K10);
    int bad = 0;
    if (!(g > eps)) bad |= BAD_GEOM;
    if (!physical_state<D::PDE, T, R>(u, R(pc.gamma))) bad |= BAD_STATE;
    if (bad) atomicOr(&s.bad, bad);
#pragma unroll
    for (int i = 0; i < D::NN; ++i) {
      R a = R(t.dphiv[q][i][0]), b = R(t.dphiv[q][i][1]);
      s.gp[q][i][0] = J11 * a - J10 * b;
      s.gp[q][i][1] = J00 * b - J01 * a;
    }
  }
  if (seed >= 0) {
#pragma unroll
    for (int c = 0; c < D::NC; ++c) {
      s.Af[q][c][0][seed] = der(f[c][0]);
      s.Af[q][c][1][seed] = der(f[c][1]);
    }
  }
}

// Face point (f, q).  dir < 0: values only; dir in [0, NC): seed u-;
// [NC, 2NC): seed u+ (interior faces); [2NC, 2NC+2): seed n~.
template <class D, class T, class R>
IFT_DEV void face_point(ElemLDS<D, R>& s, const RefTab& t, int f, int q, int dir, const PhysConst& pc) {
  constexpr int NC = D::NC;
  constexpr int NE = D::P + 1;
  const int nb = s.face[f];
  if (nb < 0 && dir >= NC && dir < 2 * NC) {
#pragma unroll
    for (int c = 0; c < NC; ++c) s.dHp[f][q][c][dir - NC] = R(0);
    return;
  }
  R tx = R(0), ty = R(0);
  T um[NC], up[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    R a = R(0), b = R(0);
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      a += R(t.L[q][k]) * s.U[t.en[f][k] * NC + c];
      b += R(t.L[q][k]) * s.Un[(f * NE + k) * NC + c];
    }
    um[c] = seedv<T, R>(a, dir == c);
    up[c] = seedv<T, R>(b, dir == NC + c);
  }
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    tx += R(t.dL[q][k]) * s.x[2 * t.en[f][k]];
    ty += R(t.dL[q][k]) * s.x[2 * t.en[f][k] + 1];
  }
  T ntx = seedv<T, R>(ty, dir == 2 * NC);
  T nty = seedv<T, R>(-tx, dir == 2 * NC + 1);
  if (nb < 0) boundary_state<D::PDE, T, R>(-nb, um, ntx, nty, pc, up);
  T H[NC];
  num_flux<D::PDE, T, R>(um, up, ntx, nty, R(pc.gamma), H);
  if (dir <= 0) {
#pragma unroll
    for (int c = 0; c < NC; ++c) s.H[f][q][c] = val(H[c]);
    if (!physical_state<D::PDE, T, R>(um, R(pc.gamma)) || !physical_state<D::PDE, T, R>(up, R(pc.gamma)))
      atomicOr(&s.bad, BAD_STATE);
  }
  if (dir >= 0) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      R d = der(H[c]);
      if (dir < NC) s.dHm[f][q][c][dir] = d;
      else if (dir < 2 * NC) s.dHp[f][q][c][dir - NC] = d;
      else s.dHn[f][q][c][dir - 2 * NC] = d;
    }
  }
}

// Phase B over the lanes of the wave.  JAC selects tangent tasks.
template <class D, class R, bool JAC>
IFT_DEV void phase_points(ElemLDS<D, R>& s, int lane, const PhysConst& pc, R kappa, R eps) {
  const RefTab& t = c_tab[D::P - 1];
  using TT = Tan<R>;
  if (!JAC) {
    constexpr int ntask = D::NQV + 3 * D::NQF + 1;
    for (int k = lane; k < ntask; k += 64) {
      if (k < D::NQV) {
        vol_point<D, R, R>(s, t, k, -1, pc, eps);
      } else if (k < D::NQV + 3 * D::NQF) {
        int r = k - D::NQV;
        face_point<D, R, R>(s, t, r / D::NQF, r % D::NQF, -1, pc);
      } else {
        R eta = eta_elem<D, R, R>(t, s.x, s.X, eps);
        R eta0 = R(0);
        for (int q = 0; q < D::NQV; ++q) {
          R K00, K01, K10, K11;
          jac2<D, R, R>(t, q, s.X, K00, K01, K10, K11);
          eta0 += R(t.wv[q]) * (K00 * K11 - K01 * K10);
        }
        s.N = kappa * (eta - R(4) * eta0);
      }
    }
  } else {
    constexpr int nvol = D::NQV * D::NC;
    constexpr int nface = 3 * D::NQF * (2 * D::NC + 2);
    constexpr int ntask = nvol + nface + D::NXE;
    for (int k = lane; k < ntask; k += 64) {
      if (k < nvol) {
        vol_point<D, TT, R>(s, t, k / D::NC, k % D::NC, pc, eps);
      } else if (k < nvol + nface) {
        int r = k - nvol;
        int dir = r % (2 * D::NC + 2);
        int pt = r / (2 * D::NC + 2);
        face_point<D, TT, R>(s, t, pt / D::NQF, pt % D::NQF, dir, pc);
      } else {
        int j = k - nvol - nface;
        TT xs[D::NXE];
#pragma unroll
        for (int i = 0; i < D::NXE; ++i) xs[i] = seedv<TT, R>(s.x[i], i == j);
        TT eta = eta_elem<D, TT, R>(t, xs, s.X, eps);
        s.dN[j] = kappa * eta.d;
        if (j == 0) {
          R eta0 = R(0);
          for (int q = 0; q < D::NQV; ++q) {
            R K00, K01, K10, K11;
            jac2<D, R, R>(t, q, s.X, K00, K01, K10, K11);
            eta0 += R(t.wv[q]) * (K00 * K11 - K01 * K10);
          }
          s.N = kappa * (eta.v - R(4) * eta0);
        }
      }
    }
  }
}

// ----------------------------------------------------------------- phase C
template <class D, class R>
IFT_DEV void phase_residual(ElemLDS<D, R>& s, int lane) {
  const RefTab& t = c_tab[D::P - 1];
  if (lane < D::NUE) {
    const int i = lane / D::NC, c = lane % D::NC;
    R r = R(0);
#pragma unroll
    for (int q = 0; q < D::NQV; ++q)
      r -= R(t.wv[q]) * (s.fv[q][c][0] * s.gp[q][i][0] + s.fv[q][c][1] * s.gp[q][i][1]);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const int k = t.nfk[i][f];
      if (k < 0) continue;
#pragma unroll
      for (int q = 0; q < D::NQF; ++q) r += R(t.wf[q] * t.L[q][k]) * s.H[f][q][c];
    }
    s.Re[lane] = r;
  }
}

// ----------------------------------------------------------------- phase D
// Column of dR_e along a state direction (dU on the element's DoFs, dUn on
// the neighbour face-trace DoFs).
template <class D, class R>
IFT_DEV void column_state(const ElemLDS<D, R>& s, const R* dU, const R* dUn, R* dR) {
  const RefTab& t = c_tab[D::P - 1];
  constexpr int NC = D::NC;
  constexpr int NE = D::P + 1;
#pragma unroll
  for (int r = 0; r < D::NUE; ++r) dR[r] = R(0);
#pragma unroll
  for (int q = 0; q < D::NQV; ++q) {
    R du[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      R a = R(0);
#pragma unroll
      for (int j = 0; j < D::NN; ++j) a += R(t.phiv[q][j]) * dU[j * NC + c];
      du[c] = a;
    }
    R w = R(t.wv[q]);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      R f0 = R(0), f1 = R(0);
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        f0 += s.Af[q][c][0][cc] * du[cc];
        f1 += s.Af[q][c][1][cc] * du[cc];
      }
      f0 *= w;
      f1 *= w;
#pragma unroll
      for (int i = 0; i < D::NN; ++i) dR[i * NC + c] -= f0 * s.gp[q][i][0] + f1 * s.gp[q][i][1];
    }
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) {
#pragma unroll
    for (int q = 0; q < D::NQF; ++q) {
      R dm[NC], dp[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        R a = R(0), b = R(0);
#pragma unroll
        for (int k = 0; k < NE; ++k) {
          a += R(t.L[q][k]) * dU[t.en[f][k] * NC + c];
          b += R(t.L[q][k]) * dUn[(f * NE + k) * NC + c];
        }
        dm[c] = a;
        dp[c] = b;
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        R h = R(0);
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) h += s.dHm[f][q][c][cc] * dm[cc] + s.dHp[f][q][c][cc] * dp[cc];
        h *= R(t.wf[q]);
#pragma unroll
        for (int k = 0; k < NE; ++k) dR[t.en[f][k] * NC + c] += R(t.L[q][k]) * h;
      }
    }
  }
}

// Column of dR_e and dN_e along a mapping direction dx on x_e.
template <class D, class R>
IFT_DEV void column_map(const ElemLDS<D, R>& s, const R* dx, R* dR, R& dNv) {
  const RefTab& t = c_tab[D::P - 1];
  constexpr int NC = D::NC;
  constexpr int NE = D::P + 1;
#pragma unroll
  for (int r = 0; r < D::NUE; ++r) dR[r] = R(0);
#pragma unroll
  for (int q = 0; q < D::NQV; ++q) {
    R J00, J01, J10, J11;
    jac2<D, R, R>(t, q, dx, J00, J01, J10, J11);
    R w = R(t.wv[q]);
#pragma unroll
    for (int i = 0; i < D::NN; ++i) {
      R a = R(t.dphiv[q][i][0]), b = R(t.dphiv[q][i][1]);
      R g0 = w * (J11 * a - J10 * b), g1 = w * (J00 * b - J01 * a);
#pragma unroll
      for (int c = 0; c < NC; ++c) dR[i * NC + c] -= s.fv[q][c][0] * g0 + s.fv[q][c][1] * g1;
    }
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) {
#pragma unroll
    for (int q = 0; q < D::NQF; ++q) {
      R tx = R(0), ty = R(0);
#pragma unroll
      for (int k = 0; k < NE; ++k) {
        tx += R(t.dL[q][k]) * dx[2 * t.en[f][k]];
        ty += R(t.dL[q][k]) * dx[2 * t.en[f][k] + 1];
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        R h = R(t.wf[q]) * (s.dHn[f][q][c][0] * ty - s.dHn[f][q][c][1] * tx);
#pragma unroll
        for (int k = 0; k < NE; ++k) dR[t.en[f][k] * NC + c] += R(t.L[q][k]) * h;
      }
    }
  }
  R a = R(0);
#pragma unroll
  for (int k = 0; k < D::NXE; ++k) a += s.dN[k] * dx[k];
  dNv = a;
}

}  // namespace ift
