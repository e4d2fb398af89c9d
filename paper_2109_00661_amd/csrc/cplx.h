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
