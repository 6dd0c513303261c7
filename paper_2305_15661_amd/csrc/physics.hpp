// Physical fluxes, numerical fluxes and boundary states, templated on the
// scalar type (double / float values, or Tan<> for one Jacobian column).
//
// Burgers: space-time flux f(u) = (u^2/2, u) of eq. (burgers) (its source
// enters at the volume points, element.hpp); local Lax-Friedrichs
// numerical flux.
// Euler: flux of the paper's eq. (euler), ideal-gas pressure; Roe's
// approximate Riemann solver with Harten's entropy fix on all four waves,
// delta = 0.1 * Roe-averaged sound speed.
// nt is the scaled outward normal (t_y, -t_x) with t = dx/ds along the edge;
// every numerical flux is homogeneous of degree one in nt.
#pragma once
#include "tangent.hpp"

namespace ift {

enum { PDE_BURGERS = 0, PDE_EULER = 1 };

template <int PDE> struct NComp;
template <> struct NComp<PDE_BURGERS> { static constexpr int value = 1; };
template <> struct NComp<PDE_EULER> { static constexpr int value = 4; };

// Problem constants seen by the device code.
struct PhysConst {
  double gamma;
  double uinf[4];   // Euler: free stream U_inf(mu); Burgers: uinf[0] on tag 1, uinf[1] on tag 3
  double src_amp;   // Burgers source s(x) = src_amp exp(src_b x) of eq. (burgers); 0: none
  double src_b;
  int all_farfield;
  int bc_st;        // Burgers: 1 = space-time data (tag 1: u = mu[0], tag 3: u = 1)
};

// f(u) as [nc][2].
template <int PDE, class T, class R>
IFT_DEV void phys_flux(const T* u, T (*f)[2], R gamma) {
  if constexpr (PDE == PDE_BURGERS) {
    f[0][0] = R(0.5) * u[0] * u[0];
    f[0][1] = u[0];
  } else {
    T rho = u[0];
    T ir = R(1) / rho;
    T vx = u[1] * ir, vy = u[2] * ir;
    T p = (gamma - R(1)) * (u[3] - R(0.5) * rho * (vx * vx + vy * vy));
    f[0][0] = u[1];
    f[0][1] = u[2];
    f[1][0] = u[1] * vx + p;
    f[1][1] = u[1] * vy;
    f[2][0] = u[2] * vx;
    f[2][1] = u[2] * vy + p;
    f[3][0] = (u[3] + p) * vx;
    f[3][1] = (u[3] + p) * vy;
  }
}

// rho > 0 and p > 0 (Euler); always true for Burgers.
template <int PDE, class T, class R>
IFT_DEV bool physical_state(const T* u, R gamma) {
  if constexpr (PDE == PDE_BURGERS) {
    return true;
  } else {
    R rho = val(u[0]);
    R p = (gamma - R(1)) * (val(u[3]) - R(0.5) * (val(u[1]) * val(u[1]) + val(u[2]) * val(u[2])) / rho);
    return (rho > R(0)) && (p > R(0));
  }
}

// |lam| with Harten's entropy fix; i2d = 1 / (2 delta).
template <class T, class R>
IFT_DEV T harten_abs(T lam, T delta, T i2d) {
  T a = tabs(lam);
  if (val(a) < val(delta)) return (lam * lam + delta * delta) * i2d;
  return a;
}

template <int PDE, class T, class R>
IFT_DEV void num_flux(const T* uL, const T* uR, T ntx, T nty, R gamma, T* H) {
  if constexpr (PDE == PDE_BURGERS) {
    T fnL = R(0.5) * uL[0] * uL[0] * ntx + uL[0] * nty;
    T fnR = R(0.5) * uR[0] * uR[0] * ntx + uR[0] * nty;
    T a = tmax(tabs(uL[0] * ntx + nty), tabs(uR[0] * ntx + nty));
    H[0] = R(0.5) * (fnL + fnR) - R(0.5) * a * (uR[0] - uL[0]);
  } else {
    const R gm1 = gamma - R(1);
    T nmag, inm;
    sqrt_rsqrt(ntx * ntx + nty * nty, nmag, inm);
    T nx = ntx * inm, ny = nty * inm;
    T rL = uL[0], rR = uR[0];
    T sL, isL, sR, isR;
    sqrt_rsqrt(rL, sL, isL);
    sqrt_rsqrt(rR, sR, isR);
    T irL = isL * isL, irR = isR * isR;
    T vxL = uL[1] * irL, vyL = uL[2] * irL, vxR = uR[1] * irR, vyR = uR[2] * irR;
    T pL = gm1 * (uL[3] - R(0.5) * rL * (vxL * vxL + vyL * vyL));
    T pR = gm1 * (uR[3] - R(0.5) * rR * (vxR * vxR + vyR * vyR));
    T qL = vxL * ntx + vyL * nty, qR = vxR * ntx + vyR * nty;   // v . n~
    T HL = (uL[3] + pL) * irL, HR = (uR[3] + pR) * irR;
    T iden = R(1) / (sL + sR);
    T rt = sL * sR;
    T ut = (sL * vxL + sR * vxR) * iden;
    T vt = (sL * vyL + sR * vyR) * iden;
    T Ht = (sL * HL + sR * HR) * iden;
    T q2 = ut * ut + vt * vt;
    T c2 = gm1 * (Ht - R(0.5) * q2);
    T ct, ict;
    sqrt_rsqrt(c2, ct, ict);
    T ic2 = ict * ict;
    T vn = ut * nx + vt * ny;
    T vtan = vt * nx - ut * ny;
    T dr = rR - rL, dp = pR - pL;
    T dvn = (vxR * nx + vyR * ny) - (vxL * nx + vyL * ny);
    T dvt = (vyR * nx - vxR * ny) - (vyL * nx - vxL * ny);
    T h2 = R(0.5) * ic2;
    T a1 = (dp - rt * ct * dvn) * h2;
    T a4 = (dp + rt * ct * dvn) * h2;
    T a2 = dr - dp * ic2;
    T a3 = rt * dvt;
    T delta = R(0.1) * ct;
    T i2d = R(5) * ict;   // 1 / (2 delta)
    T l1 = harten_abs<T, R>(vn - ct, delta, i2d) * a1;
    T l2 = harten_abs<T, R>(vn, delta, i2d);
    T l4 = harten_abs<T, R>(vn + ct, delta, i2d) * a4;
    T l2a2 = l2 * a2, l2a3 = l2 * a3;
    T d0 = l1 + l2a2 + l4;
    T d1 = l1 * (ut - ct * nx) + l2a2 * ut - l2a3 * ny + l4 * (ut + ct * nx);
    T d2 = l1 * (vt - ct * ny) + l2a2 * vt + l2a3 * nx + l4 * (vt + ct * ny);
    T d3 = l1 * (Ht - ct * vn) + l2a2 * (R(0.5) * q2) + l2a3 * vtan + l4 * (Ht + ct * vn);
    T hm = R(0.5) * nmag;
    H[0] = R(0.5) * (rL * qL + rR * qR) - hm * d0;
    H[1] = R(0.5) * (uL[1] * qL + pL * ntx + uR[1] * qR + pR * ntx) - hm * d1;
    H[2] = R(0.5) * (uL[2] * qL + pL * nty + uR[2] * qR + pR * nty) - hm * d2;
    H[3] = R(0.5) * ((uL[3] + pL) * qL + (uR[3] + pR) * qR) - hm * d3;
  }
}

// Exterior state on a boundary face with tag 1..4.
template <int PDE, class T, class R>
IFT_DEV void boundary_state(int tag, const T* um, T ntx, T nty, const PhysConst& pc, T* up) {
  constexpr int NC = NComp<PDE>::value;
  if constexpr (PDE == PDE_BURGERS) {
    if (tag == 1 || tag == 3)
      up[0] = mk<T, R>(R(pc.uinf[tag == 1 ? 0 : 1]));
    else
      up[0] = um[0];
  } else {
    if (pc.all_farfield || tag == 1) {
      for (int c = 0; c < NC; ++c) up[c] = mk<T, R>(R(pc.uinf[c]));
    } else if (tag == 2) {
      for (int c = 0; c < NC; ++c) up[c] = um[c];
    } else {
      T nmag, inm;
      sqrt_rsqrt(ntx * ntx + nty * nty, nmag, inm);
      T nx = ntx * inm, ny = nty * inm;
      T mn = um[1] * nx + um[2] * ny;
      up[0] = um[0];
      up[1] = um[1] - R(2) * mn * nx;
      up[2] = um[2] - R(2) * mn * ny;
      up[3] = um[3];
    }
  }
}

}  // namespace ift
