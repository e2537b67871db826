// Complex arithmetic for the device numerics (FP64 and FP32), written for
// gfx950.  Principal branches throughout: sqrt has its cut on the negative
// real axis with arg in (-pi/2, pi/2] (the convention of Sec. 3.1 of the
// paper for the complexified distance).
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>

#define HD __host__ __device__ __forceinline__

template <typename T>
struct cx {
  T re, im;
};
using zd = cx<double>;
using zf = cx<float>;

template <typename T> HD cx<T> C(T r, T i = T(0)) { return cx<T>{r, i}; }
template <typename T> HD cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> HD cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> HD cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <typename T> HD cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> HD cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> HD cx<T> operator*(cx<T> a, T s) { return {s * a.re, s * a.im}; }
template <typename T> HD cx<T> operator+(cx<T> a, T s) { return {a.re + s, a.im}; }
template <typename T> HD cx<T> operator-(cx<T> a, T s) { return {a.re - s, a.im}; }
template <typename T> HD cx<T> conjg(cx<T> a) { return {a.re, -a.im}; }
template <typename T> HD T abs2(cx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename T> HD T cabs_(cx<T> a) { return hypot(a.re, a.im); }
template <typename T> HD T cabs1(cx<T> a) { return fabs(a.re) + fabs(a.im); }
// fused multiply-add c + a*b
template <typename T> HD cx<T> cfma(cx<T> a, cx<T> b, cx<T> c) {
  return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}
template <typename T> HD cx<T> inv(cx<T> a) {
  // Smith's algorithm
  if (fabs(a.re) >= fabs(a.im)) {
    T r = a.im / a.re, d = a.re + a.im * r;
    return {T(1) / d, -r / d};
  } else {
    T r = a.re / a.im, d = a.re * r + a.im;
    return {r / d, T(-1) / d};
  }
}
template <typename T> HD cx<T> operator/(cx<T> a, cx<T> b) { return a * inv(b); }
template <typename T> HD cx<T> operator/(cx<T> a, T s) { return {a.re / s, a.im / s}; }

// principal square root
template <typename T> HD cx<T> csqrt_(cx<T> z) {
  T x = z.re, y = z.im;
  if (x == T(0) && y == T(0)) return {T(0), y};
  T r = hypot(x, y);
  if (x >= T(0)) {
    T t = sqrt(T(0.5) * (r + x));
    return {t, y / (T(2) * t)};
  } else {
    T t = sqrt(T(0.5) * (r - x));
    return {fabs(y) / (T(2) * t), copysign(t, y)};
  }
}
template <typename T> HD cx<T> cexp_(cx<T> z) {
  T e = exp(z.re), s, c;
  s = sin(z.im);
  c = cos(z.im);
  return {e * c, e * s};
}
template <typename T> HD cx<T> clog_(cx<T> z) { return {log(hypot(z.re, z.im)), atan2(z.im, z.re)}; }
// cos and sin of a complex argument
template <typename T> HD cx<T> ccos_(cx<T> z) {
  return {cos(z.re) * cosh(z.im), -sin(z.re) * sinh(z.im)};
}
template <typename T> HD cx<T> csin_(cx<T> z) {
  return {sin(z.re) * cosh(z.im), cos(z.re) * sinh(z.im)};
}
