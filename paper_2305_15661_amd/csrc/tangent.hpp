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
template <class R> IFT_DEV Tan<R> operator/(Tan<R> a, Tan<R> b) {
  R q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
template <class R> IFT_DEV Tan<R> operator-(Tan<R> a) { return {-a.v, -a.d}; }
template <class R> IFT_DEV Tan<R> operator+(Tan<R> a, R b) { return {a.v + b, a.d}; }
template <class R> IFT_DEV Tan<R> operator+(R a, Tan<R> b) { return {a + b.v, b.d}; }
template <class R> IFT_DEV Tan<R> operator-(Tan<R> a, R b) { return {a.v - b, a.d}; }
template <class R> IFT_DEV Tan<R> operator-(R a, Tan<R> b) { return {a - b.v, -b.d}; }
template <class R> IFT_DEV Tan<R> operator*(Tan<R> a, R b) { return {a.v * b, a.d * b}; }
template <class R> IFT_DEV Tan<R> operator*(R a, Tan<R> b) { return {a * b.v, a * b.d}; }
template <class R> IFT_DEV Tan<R> operator/(Tan<R> a, R b) { return {a.v / b, a.d / b}; }
template <class R> IFT_DEV Tan<R> operator/(R a, Tan<R> b) {
  R q = a / b.v;
  return {q, -q * b.d / b.v};
}

template <class R> IFT_DEV Tan<R> tsqrt(Tan<R> a) {
  R r = sqrt(a.v);
  return {r, a.d / (R(2) * r)};
}
IFT_DEV double tsqrt(double a) { return sqrt(a); }
IFT_DEV float tsqrt(float a) { return sqrtf(a); }

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
