// Small complex arithmetic for the gfx950 kernels (device only).
#pragma once

#include <hip/hip_runtime.h>

namespace rjsmc {

template <typename T>
struct cplx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> mk(T re, T im) {
  return cplx<T>{re, im};
}
template <typename T>
__device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename T>
__device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) {
  return {a.re - b.re, a.im - b.im};
}
template <typename T>
__device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) {
  return {s * a.re, s * a.im};
}
template <typename T>
__device__ __forceinline__ cplx<T> csq(cplx<T> a) {
  return {a.re * a.re - a.im * a.im, T(2) * a.re * a.im};
}
template <typename T>
__device__ __forceinline__ cplx<T> cdiv(cplx<T> a, cplx<T> b) {
  const T inv = T(1) / (b.re * b.re + b.im * b.im);
  return {(a.re * b.re + a.im * b.im) * inv, (a.im * b.re - a.re * b.im) * inv};
}
template <typename T>
__device__ __forceinline__ cplx<T> crcp(cplx<T> b) {
  const T inv = T(1) / (b.re * b.re + b.im * b.im);
  return {b.re * inv, -b.im * inv};
}

// 1/sqrt(x) and sqrt(x) for x > 0 (finite, normal): hardware estimate refined by two
// Goldschmidt steps (relative error a few ulp).
__device__ __forceinline__ void rsqrt_sqrt(double x, double &rs, double &sq) {
  double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  sq = g;
  rs = 2.0 * h;
}
__device__ __forceinline__ void rsqrt_sqrt(float x, float &rs, float &sq) {
  rs = __builtin_amdgcn_rsqf(x);
  sq = x * rs;
}

// 1/x for finite normal x != 0: hardware estimate and two Newton steps.
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Principal square root for Im z != 0 or Re z > 0 (z never on the closed negative
// real axis or at 0): both sqrt and its reciprocal from one refined estimate.
template <typename T>
__device__ __forceinline__ cplx<T> csqrt_fast(cplx<T> z) {
  T rs, mag;
  rsqrt_sqrt(z.re * z.re + z.im * z.im, rs, mag);
  const T w = T(0.5) * (mag + (z.re >= T(0) ? z.re : -z.re));
  T rt, t;
  rsqrt_sqrt(w, rt, t);
  const T o = T(0.5) * z.im * rt;
  if (z.re >= T(0)) return {t, o};
  return {o >= T(0) ? o : -o, z.im >= T(0) ? t : -t};
}

// Principal square root (Re >= 0), branch cut on the negative real axis.
__device__ __forceinline__ cplx<double> csqrt(cplx<double> z) {
  const double mag = sqrt(z.re * z.re + z.im * z.im);
  const double t = sqrt(0.5 * (mag + fabs(z.re)));
  if (t == 0.0) return {0.0, 0.0};
  const double o = z.im / (2.0 * t);
  return z.re >= 0.0 ? cplx<double>{t, o} : cplx<double>{fabs(o), copysign(t, z.im)};
}
__device__ __forceinline__ cplx<float> csqrt(cplx<float> z) {
  const float mag = sqrtf(z.re * z.re + z.im * z.im);
  const float t = sqrtf(0.5f * (mag + fabsf(z.re)));
  if (t == 0.0f) return {0.0f, 0.0f};
  const float o = z.im / (2.0f * t);
  return z.re >= 0.0f ? cplx<float>{t, o} : cplx<float>{fabsf(o), copysignf(t, z.im)};
}

__device__ __forceinline__ cplx<double> cexp(cplx<double> z) {
  const double e = exp(z.re);
  double s, c;
  sincos(z.im, &s, &c);
  return {e * c, e * s};
}
__device__ __forceinline__ cplx<float> cexp(cplx<float> z) {
  const float e = expf(z.re);
  float s, c;
  sincosf(z.im, &s, &c);
  return {e * c, e * s};
}

}  // namespace rjsmc
