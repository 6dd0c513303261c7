// Value + one directional derivative.  Each GPU lane that needs a column of
// a point Jacobian evaluates the point function once in this type, seeded
// along one input direction; derivatives are therefore exact (up to
// rounding) without hand-derived Jacobians.
// Kink conventions: d|x| uses sign(0) = +1; tmax(a, b) follows a on a tie.
#pragma once
#include <hip/hip_runtime.h>

#define IFT_DEV __device__ __forceinline__

template <class R>
struct Tan {
  R v, d;
};

template <class R> IFT_DEV Tan<R> operator+(Tan<R> a, Tan<R> b) { return {a.v + b.v, a.d + b.d}; }
template <class R> IFT_DEV Tan<R> operator-(Tan<R> a, Tan<R> b) { return {a.v - b.v, a.d - b.d}; }
template <class R> IFT_DEV Tan<R> operator*(Tan<R> a, Tan<R> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
// Quotients take one reciprocal of the divisor (one division per quotient
// and its derivative instead of two).
template <class R> IFT_DEV Tan<R> operator/(Tan<R> a, Tan<R> b) {
  const R r = R(1) / b.v;
  const R q = a.v * r;
  return {q, (a.d - q * b.d) * r};
}
template <class R> IFT_DEV Tan<R> operator-(Tan<R> a) { return {-a.v, -a.d}; }
template <class R> IFT_DEV Tan<R> operator+(Tan<R> a, R b) { return {a.v + b, a.d}; }
template <class R> IFT_DEV Tan<R> operator+(R a, Tan<R> b) { return {a + b.v, b.d}; }
template <class R> IFT_DEV Tan<R> operator-(Tan<R> a, R b) { return {a.v - b, a.d}; }
template <class R> IFT_DEV Tan<R> operator-(R a, Tan<R> b) { return {a - b.v, -b.d}; }
template <class R> IFT_DEV Tan<R> operator*(Tan<R> a, R b) { return {a.v * b, a.d * b}; }
template <class R> IFT_DEV Tan<R> operator*(R a, Tan<R> b) { return {a * b.v, a * b.d}; }
template <class R> IFT_DEV Tan<R> operator/(Tan<R> a, R b) {
  const R r = R(1) / b;
  return {a.v * r, a.d * r};
}
template <class R> IFT_DEV Tan<R> operator/(R a, Tan<R> b) {
  const R r = R(1) / b.v;
  const R q = a * r;
  return {q, -q * b.d * r};
}

template <class R> IFT_DEV Tan<R> tsqrt(Tan<R> a) {
  const R r = sqrt(a.v);
  return {r, a.d * (R(0.5) / r)};
}
IFT_DEV double tsqrt(double a) { return sqrt(a); }
IFT_DEV float tsqrt(float a) { return sqrtf(a); }

// sqrt(x) and 1/sqrt(x) from one square root and one division:
// d sqrt(x) = dx / (2 sqrt(x)), d x^(-1/2) = -(dx / (2 sqrt(x))) / x.
template <class R> IFT_DEV void sqrt_rsqrt(Tan<R> x, Tan<R>& s, Tan<R>& is) {
  const R r = R(1) / sqrt(x.v);
  const R h = R(0.5) * x.d * r;
  s = {x.v * r, h};
  is = {r, -h * r * r};
}
IFT_DEV void sqrt_rsqrt(double x, double& s, double& is) {
  is = 1.0 / sqrt(x);
  s = x * is;
}
IFT_DEV void sqrt_rsqrt(float x, float& s, float& is) {
  is = 1.0f / sqrtf(x);
  s = x * is;
}

template <class R> IFT_DEV Tan<R> tabs(Tan<R> a) { return a.v >= R(0) ? a : Tan<R>{-a.v, -a.d}; }
IFT_DEV double tabs(double a) { return a >= 0.0 ? a : -a; }
IFT_DEV float tabs(float a) { return a >= 0.0f ? a : -a; }

template <class R> IFT_DEV Tan<R> tmax(Tan<R> a, Tan<R> b) { return a.v >= b.v ? a : b; }
IFT_DEV double tmax(double a, double b) { return a >= b ? a : b; }
IFT_DEV float tmax(float a, float b) { return a >= b ? a : b; }

template <class R> IFT_DEV R val(Tan<R> a) { return a.v; }
IFT_DEV double val(double a) { return a; }
IFT_DEV float val(float a) { return a; }

template <class R> IFT_DEV R der(Tan<R> a) { return a.d; }
IFT_DEV double der(double) { return 0.0; }
IFT_DEV float der(float) { return 0.0f; }

// Scalar type traits: the real type underneath a (possibly tangent) scalar.
template <class T> struct RealOf { using type = T; };
template <class R> struct RealOf<Tan<R>> { using type = R; };

template <class T, class R> IFT_DEV T mk(R v) { return T(v); }
template <> IFT_DEV Tan<double> mk<Tan<double>, double>(double v) { return {v, 0.0}; }
template <> IFT_DEV Tan<float> mk<Tan<float>, float>(float v) { return {v, 0.0f}; }

template <class T, class R> IFT_DEV T seedv(R v, bool on) { return T(v); }
template <> IFT_DEV Tan<double> seedv<Tan<double>, double>(double v, bool on) { return {v, on ? 1.0 : 0.0}; }
template <> IFT_DEV Tan<float> seedv<Tan<float>, float>(float v, bool on) { return {v, on ? 1.0f : 0.0f}; }
