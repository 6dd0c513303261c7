// One DG element per 256-thread workgroup (four 64-lane waves).
//
// Discretisation (Section 2.3 of the paper, readings where it is silent):
//   R_e[i,c] = sum_faces int phi_i H_c(u-, u+, n~) ds - int grad_0 phi_i . F_c dX
//              - int phi_i S_c dX,
//   F = g f(U) G^{-T}, S = g s (eq. (p2r-flux)); s is the source of the
//   space-time Burgers problem, eq. (burgers), or zero.
// With J = dx/dxi and J0 = dX/dxi the volume integrand reduces to
// f(u) . (cof(J) grad_xi phi_i) per unit reference-triangle measure, where
// cof(J) = det(J) J^{-T} is linear in x_e in 2-D; the face term uses
// n~ = (t_y, -t_x), t = dx/ds along the edge (Nanson's relation).  The
// mapping validity test uses g = det J / det J0, and the distortion of
// eq. (dist_elem1) uses G = J J0^{-1}.
//
// Work split inside the workgroup (all data of one element staged in LDS):
//   A  load / lift the element DoFs U_e, U_e', x_e, X_e;
//   B  point physics: each thread evaluates one quadrature point, or one
//      (point, input direction) pair in tangent arithmetic, giving the point
//      fluxes and their exact point Jacobians;
//   C  residual R_e (one thread per (node, component)) and the explicit
//      element Jacobian [dR/dU_e | dR/dU_e' | dR/dx_e] (one thread per
//      entry), assembled from the point Jacobians and the basis tables.
#pragma once
#include <type_traits>

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
  double wl[6][3][3];    // wf[q] * L[q][nfk[i][f]], 0 where node i is not on face f  [i][f][q]
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
  static constexpr int NE = P_ + 1;          // nodes per edge
  static constexpr int NUE = NN * NC;
  static constexpr int NUN = 3 * (P_ + 1) * NC;
  static constexpr int NXE = 2 * NN;
  static constexpr int NDIR = NUE + NUN + NXE;  // columns of the explicit Jacobian
};

constexpr int NTHR = 256;

enum { BAD_GEOM = 1, BAD_STATE = 2 };

// Source of eq. (burgers) at the volume points, present for Burgers only
// (an empty base otherwise): with s_q = s(x_q) at the mapped point x_q,
//   src[q][0]      = det J s_q                 (the source integrand, S = g s
//                                               per unit reference measure),
//   src[q][1 + ab] = s_q d det J / dJ_ab       (ab = 2a + b, J_ab = dx_a/dxi_b),
//   src[q][5]      = b det J s_q               (through the position, ds/dx = b s).
template <class D, class R, bool = (D::PDE == PDE_BURGERS)>
struct PtsSrc {
  R src[D::NQV][6];
};
template <class D, class R>
struct PtsSrc<D, R, false> {};

template <class R>
IFT_DEV R exp_r(R v) {
  if constexpr (std::is_same<R, float>::value) return expf(v);
  else return exp(v);
}

// Point data of one element: fluxes and exact point Jacobians at the
// volume and face quadrature points, the distortion and its gradient, and
// the validity flags.  This is what the point-physics kernel hands to the
// assembly kernel (a plain copy through global memory).
template <class D, class R>
struct Pts : PtsSrc<D, R> {
  R fv[D::NQV][D::NC][2];          // f(u_q)
  R Af[D::NQV][D::NC][2][D::NC];   // df/du at volume points: [q][c][dim][c']
  R gp[D::NQV][D::NN][2];          // cof(J) grad_xi phi_i
  R H[3][D::NQF][D::NC];           // numerical flux at face points
  R dHm[3][D::NQF][D::NC][D::NC];  // dH/du- (boundary state dependence included)
  R dHp[3][D::NQF][D::NC][D::NC];  // dH/du+ (interior faces)
  R dHn[3][D::NQF][D::NC][2];      // dH/dn~ (wall state dependence included)
  R dN[D::NXE];                    // dN_e/dx_e
  R dv[64];                        // EQ kernels: distortion row of the projection, dN_e Psi_e (entries j < m)
  R N;
  int bad;
  int pad_;
};


template <class D, class R>
struct ElemLDS {
  RefTab tab;
  R U[D::NUE];
  R Un[D::NUN];
  R x[D::NXE];
  R X[D::NXE];
  int face[3];
  alignas(16) Pts<D, R> p;   // 16-byte aligned: copied out in 16-byte words where its size allows
  R Re[D::NUE];
  R deta[D::NQV][5];   // per volume point: distortion integrand and its J-gradient
  R eta_ref;           // distortion of the reference element X_e (precomputed per element; the loaders fill it)
  double cf[2][64];    // lift coefficients (w, tau), zero-padded, one vector per loading wave
};

// With the explicit element Jacobian (the assembly kernel that writes its
// blocks from LDS); the point kernels leave it out (13.8 KB per element in
// FP64 for Euler P2, which would otherwise bound their occupancy by LDS).
template <class D, class R>
struct ElemLDSJx : ElemLDS<D, R> {
  R Jx[D::NUE][D::NDIR];   // [dR/dU_e | dR/dU_e' | dR/dx_e]
};

// Copies an object of type T with NT threads in the widest words (16, 8 or
// 4 bytes) that its size and ALIGN, the alignment both ends guarantee,
// allow: a fixed trip count, and every load of a thread issued before its
// first store, so the copy costs one memory latency instead of one per word
// (and fewer, wider accesses).
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
template <class T, int NT, int ALIGN = alignof(T)>
IFT_DEV void copy_obj(T* dst, const T* src, int tid) {
  static_assert(sizeof(T) % 4 == 0 && ALIGN >= 4, "whole 4-byte words");
  using W8 = typename std::conditional<sizeof(T) % 8 == 0 && ALIGN >= 8, unsigned long long, unsigned>::type;
  using W = typename std::conditional<sizeof(T) % 16 == 0 && ALIGN >= 16, u32x4, W8>::type;
  constexpr int nw = (int)(sizeof(T) / sizeof(W)), it = (nw + NT - 1) / NT;
  W* d = reinterpret_cast<W*>(dst);
  const W* s = reinterpret_cast<const W*>(src);
  W v[it];
#pragma unroll
  for (int i = 0; i < it; ++i)
    if (tid + i * NT < nw) v[i] = s[tid + i * NT];
#pragma unroll
  for (int i = 0; i < it; ++i)
    if (tid + i * NT < nw) d[tid + i * NT] = v[i];
}

template <class D, class R, int NT>
IFT_DEV void load_tab(ElemLDS<D, R>& s, int tid) {
  copy_obj<RefTab, NT>(&s.tab, &c_tab[D::P - 1], tid);
}

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

// Distortion integrand at volume point q, eq. (dist_elem1) with 2/d = 1:
// w_q det J0 (|G|_F^2 / max(g, eps))^2 with G = J J0^{-1}, g = det J / det J0.
template <class D, class T, class R>
IFT_DEV T eta_point(const RefTab& t, int q, T J00, T J01, T J10, T J11, const R* X, R eps) {
  R K00, K01, K10, K11;
  jac2<D, R, R>(t, q, X, K00, K01, K10, K11);
  R dK = K00 * K11 - K01 * K10;
  const R idK = R(1) / dK;
  R i00 = K11 * idK, i01 = -K01 * idK, i10 = -K10 * idK, i11 = K00 * idK;
  T G00 = J00 * i00 + J01 * i10, G01 = J00 * i01 + J01 * i11;
  T G10 = J10 * i00 + J11 * i10, G11 = J10 * i01 + J11 * i11;
  T nG2 = G00 * G00 + G01 * G01 + G10 * G10 + G11 * G11;
  T g = (J00 * J11 - J01 * J10) * idK;
  T mx = val(g) >= eps ? g : mk<T, R>(eps);
  T r = nG2 / mx;
  return (R(t.wv[q]) * dK) * (r * r);
}

// eta_e and, for seed >= 0, its derivative along mapping coordinate `seed`
// of x_e (node seed/2, component seed%2): only J carries a tangent, and it
// is sparse: dJ[a][b] = d phi_node / d xi_b for the seeded component a.
template <class D, class R>
IFT_DEV Tan<R> eta_elem(const RefTab& t, const R* x, const R* X, R eps, int seed) {
  using TT = Tan<R>;
  TT eta = {R(0), R(0)};
  const int kn = seed >> 1, ka = seed & 1;
#pragma unroll 1
  for (int q = 0; q < D::NQV; ++q) {
    R J00, J01, J10, J11;
    jac2<D, R, R>(t, q, x, J00, J01, J10, J11);
    R d0 = R(0), d1 = R(0);
    if (seed >= 0) {
      d0 = R(t.dphiv[q][kn][0]);
      d1 = R(t.dphiv[q][kn][1]);
    }
    TT a00 = {J00, ka == 0 ? d0 : R(0)}, a01 = {J01, ka == 0 ? d1 : R(0)};
    TT a10 = {J10, ka == 1 ? d0 : R(0)}, a11 = {J11, ka == 1 ? d1 : R(0)};
    eta = eta + eta_point<D, TT, R>(t, q, a00, a01, a10, a11, X, eps);
  }
  return eta;
}

// Distortion integrand at volume point q and its gradient with respect to
// J = dx/dxi, in plain arithmetic: out[0] = w_q det J0 (|G|_F^2 / max(g,
// eps))^2 and out[1 + 2a + b] = its derivative along J[a][b].  With
// r = |G|^2 / max(g, eps): d|G|^2/dJ = 2 G J0^{-T}, dg/dJ = cof(J) / det J0
// (through the max only where g >= eps, as the tangent form).
template <class D, class R>
IFT_DEV void eta_point_grad(const RefTab& t, int q, const R* x, const R* X, R eps, R* out) {
  R J00, J01, J10, J11, K00, K01, K10, K11;
  jac2<D, R, R>(t, q, x, J00, J01, J10, J11);
  jac2<D, R, R>(t, q, X, K00, K01, K10, K11);
  const R dK = K00 * K11 - K01 * K10;
  const R idK = R(1) / dK;
  const R i00 = K11 * idK, i01 = -K01 * idK, i10 = -K10 * idK, i11 = K00 * idK;
  const R G00 = J00 * i00 + J01 * i10, G01 = J00 * i01 + J01 * i11;
  const R G10 = J10 * i00 + J11 * i10, G11 = J10 * i01 + J11 * i11;
  const R nG2 = G00 * G00 + G01 * G01 + G10 * G10 + G11 * G11;
  const R g = (J00 * J11 - J01 * J10) * idK;
  const bool act = g >= eps;
  const R mx = act ? g : eps;
  const R imx = R(1) / mx;
  const R r = nG2 * imx;
  const R c = R(t.wv[q]) * dK;
  out[0] = c * (r * r);
  const R s = R(2) * c * r * imx;           // d eta / d |G|^2
  const R sg = act ? -s * r * idK : R(0);   // d eta / d det J
  out[1] = R(2) * s * (G00 * i00 + G01 * i01) + sg * J11;
  out[2] = R(2) * s * (G00 * i10 + G01 * i11) - sg * J10;
  out[3] = R(2) * s * (G10 * i00 + G11 * i01) - sg * J01;
  out[4] = R(2) * s * (G10 * i10 + G11 * i11) + sg * J00;
}

template <class D, class R>
IFT_DEV R eta_reference(const RefTab& t, const R* X) {
  // at x = X: G = I, |G|_F^2 = 2, g = 1, so the integrand is 4
  R a = R(0);
#pragma unroll
  for (int q = 0; q < D::NQV; ++q) {
    R K00, K01, K10, K11;
    jac2<D, R, R>(t, q, X, K00, K01, K10, K11);
    a += R(t.wv[q]) * (K00 * K11 - K01 * K10);
  }
  return R(4) * a;
}

// Volume point q: state, flux, cof(J) grad phi; seed = component seeded in
// tangent mode (-1: none).  Returns the flux Jacobian column in Af.
template <class D, class T, class R, class S>
IFT_DEV void vol_point(const RefTab& t, S& s, int q, int seed, const PhysConst& pc, R eps) {
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
      s.p.fv[q][c][0] = val(f[c][0]);
      s.p.fv[q][c][1] = val(f[c][1]);
    }
    R J00, J01, J10, J11, K00, K01, K10, K11;
    jac2<D, R, R>(t, q, s.x, J00, J01, J10, J11);
    jac2<D, R, R>(t, q, s.X, K00, K01, K10, K11);
    R g = (J00 * J11 - J01 * J10) / (K00 * K11 - K01 * K10);
    int bad = 0;
    if (!(g > eps)) bad |= BAD_GEOM;
    if (!physical_state<D::PDE, T, R>(u, R(pc.gamma))) bad |= BAD_STATE;
    if (bad) atomicOr(&s.p.bad, bad);
#pragma unroll
    for (int i = 0; i < D::NN; ++i) {
      R a = R(t.dphiv[q][i][0]), b = R(t.dphiv[q][i][1]);
      s.p.gp[q][i][0] = J11 * a - J10 * b;
      s.p.gp[q][i][1] = J00 * b - J01 * a;
    }
    if constexpr (D::PDE == PDE_BURGERS) {
      // source at the mapped position x_q = sum_j x_j phi_j(xi_q)
      R xq = R(0);
#pragma unroll
      for (int j = 0; j < D::NN; ++j) xq += R(t.phiv[q][j]) * s.x[2 * j];
      const R sq = pc.src_amp != 0.0 ? R(pc.src_amp) * exp_r<R>(R(pc.src_b) * xq) : R(0);
      const R dJ = J00 * J11 - J01 * J10;
      s.p.src[q][0] = dJ * sq;
      s.p.src[q][1] = sq * J11;
      s.p.src[q][2] = -(sq * J10);
      s.p.src[q][3] = -(sq * J01);
      s.p.src[q][4] = sq * J00;
      s.p.src[q][5] = R(pc.src_b) * s.p.src[q][0];
    }
  }
  if constexpr (!std::is_same<T, R>::value) {
    if (seed >= 0) {
#pragma unroll
      for (int c = 0; c < D::NC; ++c) {
        s.p.Af[q][c][0][seed] = der(f[c][0]);
        s.p.Af[q][c][1][seed] = der(f[c][1]);
      }
    }
  }
}

// Face point (f, q).  dir < 0: values only; dir in [0, NC): seed u-;
// [NC, 2NC): seed u+ (interior faces); [2NC, 2NC+2): seed n~.
template <class D, class T, class R, class S>
IFT_DEV void face_point(const RefTab& t, S& s, int f, int q, int dir, const PhysConst& pc) {
  constexpr int NC = D::NC;
  constexpr int NE = D::NE;
  const int nb = s.face[f];
  if constexpr (!std::is_same<T, R>::value) {
    if (nb < 0 && dir >= NC && dir < 2 * NC) {
#pragma unroll
      for (int c = 0; c < NC; ++c) s.p.dHp[f][q][c][dir - NC] = R(0);
      return;
    }
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
    for (int c = 0; c < NC; ++c) s.p.H[f][q][c] = val(H[c]);
    if (!physical_state<D::PDE, T, R>(um, R(pc.gamma)) || !physical_state<D::PDE, T, R>(up, R(pc.gamma)))
      atomicOr(&s.p.bad, BAD_STATE);
  }
  if constexpr (!std::is_same<T, R>::value) {
    if (dir >= 0) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        R d = der(H[c]);
        if (dir < NC) s.p.dHm[f][q][c][dir] = d;
        else if (dir < 2 * NC) s.p.dHp[f][q][c][dir - NC] = d;
        else s.p.dHn[f][q][c][dir - 2 * NC] = d;
      }
    }
  }
}

// Number of phase-B tasks per element.
template <class D, bool JAC>
constexpr int n_point_tasks() {
  return JAC ? D::NQV * D::NC + 3 * D::NQF * (2 * D::NC + 2) + D::NQV : D::NQV + 3 * D::NQF + 1;
}

// Phase B: thread `tid` runs task `tid` (every launch has at least as many
// threads as tasks; a single guarded task, not a loop, keeps the compiler
// from hoisting the table loads of all task kinds at once).  JAC selects
// tangent tasks.
template <class D, class R, bool JAC>
IFT_DEV void phase_points(ElemLDS<D, R>& s, int tid, const PhysConst& pc, R kappa, R eps) {
  using TT = Tan<R>;
  if (!JAC) {
    constexpr int ntask = n_point_tasks<D, false>();
    if (tid < ntask) {
      const int k = tid;
      if (k < D::NQV) {
        vol_point<D, R, R>(s.tab, s, k, -1, pc, eps);
      } else if (k < D::NQV + 3 * D::NQF) {
        int r = k - D::NQV;
        face_point<D, R, R>(s.tab, s, r / D::NQF, r % D::NQF, -1, pc);
      } else {
        Tan<R> eta = eta_elem<D, R>(s.tab, s.x, s.X, eps, -1);
        s.p.N = kappa * (eta.v - s.eta_ref);
      }
    }
  } else {
    constexpr int nvol = D::NQV * D::NC;
    constexpr int nface = 3 * D::NQF * (2 * D::NC + 2);
    constexpr int ntask = n_point_tasks<D, true>();
    if (tid < ntask) {
      int k = tid;
      if constexpr (nface >= 64) {
        // wave 0: faces, then the distortion tasks; wave 1: the other
        // faces, then the volume tasks (each wave's lanes run their kinds of
        // task one after the other, so the two waves' chains are balanced)
        constexpr int f0 = 64 - D::NQV;
        if (tid >= f0 && tid < 64) k = nface + nvol + (tid - f0);
        else if (tid >= 64 && tid < 64 + nface - f0) k = tid - 64 + f0;
        else if (tid >= 64 + nface - f0) k = nface + (tid - 64 - (nface - f0));
      }
      // face tasks first so that whole waves run the (heavier) face path
      if (k < nface) {
        int dir = k % (2 * D::NC + 2);
        int pt = k / (2 * D::NC + 2);
        face_point<D, TT, R>(s.tab, s, pt / D::NQF, pt % D::NQF, dir, pc);
      } else if (k < nface + nvol) {
        const int r = k - nface;
        vol_point<D, TT, R>(s.tab, s, r / D::NC, r % D::NC, pc, eps);
      } else {
        // distortion: one volume point per task, gathered by phase_distortion
        eta_point_grad<D, R>(s.tab, k - nvol - nface, s.x, s.X, eps, s.deta[k - nvol - nface]);
      }
    }
  }
}

// Phase B with Jacobians for two elements in a 256-thread block, used when
// one element has at least 64 face tasks (four-component P2).  The 2 x nface
// face tasks fill waves 0-2 evenly; wave 3 runs the 2 x NQV*NC volume tasks
// and then the 2 x NQV distortion tasks.  No wave runs both the face and the
// volume path, which the one-element layout cannot avoid.  pc_of(h) gives
// the physical constants of element h (the two may belong to different
// instances of a batch).
template <class D>
constexpr bool pair_layout() {
  constexpr int nface = 3 * D::NQF * (2 * D::NC + 2), nvol = D::NQV * D::NC;
  return nface >= 64 && (2 * nface) % 3 == 0 && 2 * nface / 3 <= 64 && 2 * (nvol + D::NQV) <= 64;
}

template <class D, class R, class PC>
IFT_DEV void phase_points_pair(ElemLDS<D, R>* s, int tid, const PC& pc_of, R eps) {
  static_assert(pair_layout<D>(), "two-element layout");
  using TT = Tan<R>;
  constexpr int nvol = D::NQV * D::NC;
  constexpr int nface = 3 * D::NQF * (2 * D::NC + 2);
  constexpr int fw = 2 * nface / 3;   // face lanes per wave
  const int w = tid >> 6, l = tid & 63;
  if (w < 3) {
    if (l < fw) {
      const int g = w * fw + l, h = g / nface, k = g % nface;
      const int dir = k % (2 * D::NC + 2), pt = k / (2 * D::NC + 2);
      face_point<D, TT, R>(s[h].tab, s[h], pt / D::NQF, pt % D::NQF, dir, pc_of(h));
    }
  } else if (l < 2 * nvol) {
    const int h = l / nvol, r = l % nvol;
    vol_point<D, TT, R>(s[h].tab, s[h], r / D::NC, r % D::NC, pc_of(h), eps);
  } else if (l < 2 * nvol + 2 * D::NQV) {
    const int h = (l - 2 * nvol) / D::NQV, q = (l - 2 * nvol) % D::NQV;
    eta_point_grad<D, R>(s[h].tab, q, s[h].x, s[h].X, eps, s[h].deta[q]);
  }
}

// After phase B with Jacobians (and a barrier): N_e and dN_e/dx_e from the
// per-point distortion terms, J = sum_k x_k grad_xi phi_k.
template <class D, class R>
IFT_DEV void phase_distortion(ElemLDS<D, R>& s, int tid, R kappa) {
  if (tid < D::NXE) {
    const int k = tid >> 1, a = tid & 1;
    R v = R(0);
#pragma unroll
    for (int q = 0; q < D::NQV; ++q)
      v += s.deta[q][1 + 2 * a] * R(s.tab.dphiv[q][k][0]) + s.deta[q][2 + 2 * a] * R(s.tab.dphiv[q][k][1]);
    s.p.dN[tid] = kappa * v;
  } else if (tid == D::NXE) {
    R eta = R(0);
#pragma unroll
    for (int q = 0; q < D::NQV; ++q) eta += s.deta[q][0];
    s.p.N = kappa * (eta - s.eta_ref);
  }
}

// ----------------------------------------------------------------- phase C
template <class D, class R, class P>
IFT_DEV R residual_entry_p(const P& p, const RefTab& t, int r) {
  const int i = r / D::NC, c = r % D::NC;
  R v = R(0);
#pragma unroll
  for (int q = 0; q < D::NQV; ++q) v -= R(t.wv[q]) * (p.fv[q][c][0] * p.gp[q][i][0] + p.fv[q][c][1] * p.gp[q][i][1]);
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int k = t.nfk[i][f];
    if (k < 0) continue;
#pragma unroll
    for (int q = 0; q < D::NQF; ++q) v += R(t.wf[q] * t.L[q][k]) * p.H[f][q][c];
  }
  if constexpr (D::PDE == PDE_BURGERS) {
#pragma unroll
    for (int q = 0; q < D::NQV; ++q) v -= R(t.wv[q] * t.phiv[q][i]) * p.src[q][0];
  }
  return v;
}

// Source part of dR/dx_e[i][2 k + a] (Burgers): through det J and through
// the position, -sum_q w_q phi_i (s dJ/dJ_a. . grad_xi phi_k + [a = 0] b det J s phi_k).
template <class D, class R, class P>
IFT_DEV R source_dx(const P& p, const RefTab& t, int i, int k, int a) {
  R v = R(0);
  if constexpr (D::PDE == PDE_BURGERS) {
#pragma unroll
    for (int q = 0; q < D::NQV; ++q) {
      R d = p.src[q][1 + 2 * a] * R(t.dphiv[q][k][0]) + p.src[q][2 + 2 * a] * R(t.dphiv[q][k][1]);
      if (a == 0) d += p.src[q][5] * R(t.phiv[q][k]);
      v -= R(t.wv[q] * t.phiv[q][i]) * d;
    }
  }
  return v;
}

template <class D, class R>
IFT_DEV R residual_entry(const ElemLDS<D, R>& s, int r) {
  return residual_entry_p<D, R>(s.p, s.tab, r);
}

// Entry (r, col) of [dR/dU_e | dR/dU_e' | dR/dx_e] from the point Jacobians.
template <class D, class R>
IFT_DEV R jacobian_entry(const ElemLDS<D, R>& s, int r, int col) {
  const RefTab& t = s.tab;
  constexpr int NC = D::NC;
  const int i = r / NC, c = r % NC;
  R v = R(0);
  if (col < D::NUE) {
    // d/dU_e[j, c']: volume through the flux Jacobian, faces through dH/du-
    const int j = col / NC, cc = col % NC;
#pragma unroll
    for (int q = 0; q < D::NQV; ++q)
      v -= R(t.wv[q] * t.phiv[q][j]) * (s.p.Af[q][c][0][cc] * s.p.gp[q][i][0] + s.p.Af[q][c][1][cc] * s.p.gp[q][i][1]);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const int ki = t.nfk[i][f], kj = t.nfk[j][f];
      if (ki < 0 || kj < 0) continue;
#pragma unroll
      for (int q = 0; q < D::NQF; ++q) v += R(t.wf[q] * t.L[q][ki] * t.L[q][kj]) * s.p.dHm[f][q][c][cc];
    }
  } else if (col < D::NUE + D::NUN) {
    // d/dU_e'[f, k, c']: only faces containing node i, through dH/du+
    const int cn = col - D::NUE;
    const int f = cn / (D::NE * NC), kn = (cn / NC) % D::NE, cc = cn % NC;
    const int ki = t.nfk[i][f];
    if (ki >= 0) {
#pragma unroll
      for (int q = 0; q < D::NQF; ++q) v += R(t.wf[q] * t.L[q][ki] * t.L[q][kn]) * s.p.dHp[f][q][c][cc];
    }
  } else {
    // d/dx_e[k, a]: cof(J) grad phi_i is linear in x_e; n~ is linear in x_e
    const int xx = col - D::NUE - D::NUN;
    const int k = xx >> 1, a = xx & 1;
#pragma unroll
    for (int q = 0; q < D::NQV; ++q) {
      const R K = R(t.dphiv[q][k][0] * t.dphiv[q][i][1] - t.dphiv[q][k][1] * t.dphiv[q][i][0]);
      v += (a == 0 ? -s.p.fv[q][c][1] : s.p.fv[q][c][0]) * (R(t.wv[q]) * K);
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const int ki = t.nfk[i][f], kk = t.nfk[k][f];
      if (ki < 0 || kk < 0) continue;
#pragma unroll
      for (int q = 0; q < D::NQF; ++q)
        v += R(t.wf[q] * t.L[q][ki] * t.dL[q][kk]) * (a == 0 ? -s.p.dHn[f][q][c][1] : s.p.dHn[f][q][c][0]);
    }
    v += source_dx<D, R>(s.p, t, i, k, a);
  }
  return v;
}

// Blocked entries of the element Jacobian for four state components: the
// four columns (node j, components 0..3) of row r share the basis and
// geometry factors, and the four flux-Jacobian components are contiguous.
// dR/dU_e[r][4 j + cc]: volume terms through df/du, faces through dH/du-.
template <class D, class R>
IFT_DEV void jac_u4(const RefTab& t, const Pts<D, R>& p, int r, int j, R* out) {
  static_assert(D::NC == 4, "four state components");
  const int i = r / 4, c = r % 4;
  R v[4] = {R(0), R(0), R(0), R(0)};
#pragma unroll
  for (int q = 0; q < D::NQV; ++q) {
    const R w = R(t.wv[q] * t.phiv[q][j]);
    const R g0 = p.gp[q][i][0] * w, g1 = p.gp[q][i][1] * w;
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) v[cc] -= p.Af[q][c][0][cc] * g0 + p.Af[q][c][1][cc] * g1;
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int ki = t.nfk[i][f], kj = t.nfk[j][f];
    if (ki < 0 || kj < 0) continue;
#pragma unroll
    for (int q = 0; q < D::NQF; ++q) {
      const R w = R(t.wf[q] * t.L[q][ki] * t.L[q][kj]);
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) v[cc] += w * p.dHm[f][q][c][cc];
    }
  }
#pragma unroll
  for (int cc = 0; cc < 4; ++cc) out[cc] = v[cc];
}

// dR/dU_e'[r][4 (NE f + kn) + cc]: faces of node i through dH/du+.
template <class D, class R>
IFT_DEV void jac_un4(const RefTab& t, const Pts<D, R>& p, int r, int f, int kn, R* out) {
  const int i = r / 4, c = r % 4;
  R v[4] = {R(0), R(0), R(0), R(0)};
  const int ki = t.nfk[i][f];
  if (ki >= 0) {
#pragma unroll
    for (int q = 0; q < D::NQF; ++q) {
      const R w = R(t.wf[q] * t.L[q][ki] * t.L[q][kn]);
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) v[cc] += w * p.dHp[f][q][c][cc];
    }
  }
#pragma unroll
  for (int cc = 0; cc < 4; ++cc) out[cc] = v[cc];
}

// dR/dx_e[r][2 kn + a], a = 0, 1: cof(J) grad phi_i and n~ are linear in x_e.
template <class D, class R>
IFT_DEV void jac_x2(const RefTab& t, const Pts<D, R>& p, int r, int kn, R* out) {
  const int i = r / D::NC, c = r % D::NC;
  R v0 = R(0), v1 = R(0);
#pragma unroll
  for (int q = 0; q < D::NQV; ++q) {
    const R K = R(t.wv[q] * (t.dphiv[q][kn][0] * t.dphiv[q][i][1] - t.dphiv[q][kn][1] * t.dphiv[q][i][0]));
    v0 -= p.fv[q][c][1] * K;
    v1 += p.fv[q][c][0] * K;
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int ki = t.nfk[i][f], kk = t.nfk[kn][f];
    if (ki < 0 || kk < 0) continue;
#pragma unroll
    for (int q = 0; q < D::NQF; ++q) {
      const R w = R(t.wf[q] * t.L[q][ki] * t.dL[q][kk]);
      v0 -= w * p.dHn[f][q][c][1];
      v1 += w * p.dHn[f][q][c][0];
    }
  }
  out[0] = v0 + source_dx<D, R>(p, t, i, kn, 0);
  out[1] = v1 + source_dx<D, R>(p, t, i, kn, 1);
}

template <class D, class R, bool JAC, class S>
IFT_DEV void phase_assemble(S& s, int tid) {
  for (int r = tid; r < D::NUE; r += NTHR) s.Re[r] = residual_entry<D, R>(s, r);
  if constexpr (JAC) {
    for (int e = tid; e < D::NUE * D::NDIR; e += NTHR) {
      const int r = e / D::NDIR, col = e % D::NDIR;
      s.Jx[r][col] = jacobian_entry<D, R>(s, r, col);
    }
  }
}

}  // namespace ift
