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

// sqrt(x) and 1/(2 sqrt(x)) for x > 0 (finite, normal) from the hardware reciprocal-
// square-root estimate y = (1 + e)/sqrt(x) (|e| < 2^-24): with g = x y and
// v = 1 - g y = 1 - (1 + e)^2, sqrt(x) = g (1 - v)^(-1/2) and 1/(2 sqrt(x)) =
// (y/2) (1 - v)^(-1/2), the factor taken to second order in v, 1 + v/2 + 3v^2/8 (one
// Goldschmidt step of third order; the remainder 5v^3/16 is below 2^-70): relative error
// within about an ulp.  Without hrs (unused) it costs five operations besides the estimate.
__device__ __forceinline__ void sqrt_hrsqrt(double x, double &sq, double &hrs) {
  const double y = __builtin_amdgcn_rsq(x);
  const double g = x * y;
  const double v = fma(-g, y, 1.0);
  const double q = v * fma(v, 0.375, 0.5);
  sq = fma(g, q, g);
  const double h = 0.5 * y;
  hrs = fma(h, q, h);
}
__device__ __forceinline__ void sqrt_hrsqrt(float x, float &sq, float &hrs) {
  // the estimate is good to ~2^-23; one Goldschmidt step brings both to about an ulp
  const float y = __builtin_amdgcn_rsqf(x);
  const float g = x * y, h = 0.5f * y;
  const float r = fmaf(-g, h, 0.5f);
  sq = fmaf(g, r, g);
  hrs = fmaf(h, r, h);
}

// 1/x for finite normal x != 0: the hardware estimate r and one third-order step,
// r (1 + e + e^2) with e = 1 - x r (1/x = r / (1 - e); the remainder e^3 is below 2^-70).
__device__ __forceinline__ double fast_rcp(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}
__device__ __forceinline__ float fast_rcp(float x) {
  const float r = __builtin_amdgcn_rcpf(x);   // estimate, then one Newton step
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Principal square root for Im z != 0 or Re z > 0 (z never on the closed negative
// real axis or at 0): both sqrt and its reciprocal from one refined estimate.
template <typename T>
__device__ __forceinline__ cplx<T> csqrt_fast(cplx<T> z) {
  T mag, hm;
  sqrt_hrsqrt(z.re * z.re + z.im * z.im, mag, hm);
  const T w = T(0.5) * (mag + fabs(z.re));
  T t, ht;
  sqrt_hrsqrt(w, t, ht);
  const T oa = fabs(z.im) * ht;   // |Im z| / (2 t)
  const bool right = z.re >= T(0);
  return {right ? t : oa, copysign(right ? oa : t, z.im)};
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

// Constants of the table reductions of the FP64 exponentials: 1/ln 2; ln 2 as a double and
// the remainder (the weights' exponential subtracts both, the propagation factors' the
// first only); 2/pi; pi/2 as a double; and 1/n!.
namespace detail {
constexpr double kInvLn2 = 0x1.71547652b82fep+0;
constexpr double kLn2Hi = 0x1.62e42fefa39efp-1, kLn2Lo = 0x1.abc9e3b39803fp-56;
constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
constexpr double kPio2A = 0x1.921fb54442d18p+0;
// 1/n! for n = 0..6 (every n! here is exact in double: one rounding per entry)
constexpr double kInvFact[7] = {1.0, 1.0, 1.0 / 2.0, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0};
}  // namespace detail

// 1/6 and 1/24, the two constants the polynomials of cexp_tab share.  Each of three polynomial
// steps has two constants that are not inline operands, and an instruction takes at most
// one from a scalar register, so the other is copied into a vector register at every
// evaluation unless it already lives in one: exp_consts() puts both there, opaque to the
// compiler, so that a loop of evaluations keeps them (two register pairs) instead.
struct ExpConsts {
  double c6, c24;
};
__device__ __forceinline__ ExpConsts exp_consts() {
  double c6 = detail::kInvFact[3], c24 = detail::kInvFact[4];
  asm volatile("" : "+v"(c6), "+v"(c24));
  return {c6, c24};
}

// exp(z) for the propagation factors in FP64, Re z <= 0, with two tables in LDS:
// phase[j] = (cos, sin)(j pi/128) and e2[j] = 2^(j/256), j = 0..255.  With
//   k = round(256 x / ln 2), r = x - k ln2/256 (|r| <= ln2/512),
//   j = round(128 y / pi),   d = y - j pi/128  (|d| <= pi/256),
//   exp(x + iy) = 2^floor(k/256) e2[k mod 256] e^r phase[j mod 256] (cos d + i sin d),
// and Taylor polynomials of degree 4 (e^r), 5 (sin d) and 6 (cos d), whose remainders
// are below 4e-17, 9e-18 and 2e-20.  ln 2 and pi/2 enter the reductions as one double
// each: their rounding errors (2.3e-17 and 6.1e-17), times k/256 and j/64, put r and d
// off by at most 3.4e-17 |x| and 3.9e-17 |y|, so the relative error of exp(z) is a few
// ulp plus 4e-17 (|x| + |y|) <= 6e-17 |z|: a few ulp while |z| is of order one, 2.3e-15
// at |z| = 40, where a propagation factor exp(-2 h u) is below 4e-7 (|Im u| <= 2.5 Re u
// for every Cole-Cole layer with m <= 1, so |y| <= 2.5 |x|), and 1.4e-13 at the clamp
// below (|x| = 1000, |y| <= 2500), where it is below e^-1000.  k and
// j are rounded by adding 1.5 2^52, which leaves them as integers in the low word.
// Re z < -1000 gives 0; a NaN real part is clamped too (the recursion still propagates
// it through u), a NaN imaginary part gives NaN.  kc: the shared polynomial constants
// (from exp_consts() where the call sits in a loop).
__device__ __forceinline__ cplx<double> cexp_tab(cplx<double> z, const cplx<double> *phase,
                                                 const double *e2,
                                                 ExpConsts kc = {detail::kInvFact[3], detail::kInvFact[4]}) {
  using namespace detail;
  constexpr double kRound = 0x1.8p52;
  const double x = fmax(z.re, -1000.0);
  const double kr = fma(x, 256.0 * kInvLn2, kRound);
  const int ki = __double2loint(kr);
  const double kx = kr - kRound;
  const double r = fma(kx, -(kLn2Hi / 256.0), x);
  double p = fma(r, kInvFact[4], kc.c6);
  p = fma(p, r, kInvFact[2]);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  const double e = ldexp(p * e2[ki & 255], ki >> 8);   // ki >> 8 = floor(ki / 256)

  const double jr = fma(z.im, 64.0 * kTwoOverPi, kRound);
  const int ji = __double2loint(jr);
  const double jy = jr - kRound;
  const double d = fma(jy, -(kPio2A / 64.0), z.im);
  const double x2 = -(d * d);
  const double sd = fma(d * x2, fma(x2, kInvFact[5], kc.c6), d);
  double C = fma(x2, kInvFact[6], kc.c24);
  C = fma(C, x2, kInvFact[2]);
  const double cd = fma(x2, C, 1.0);
  const cplx<double> t = phase[ji & 255];
  return {e * fma(t.re, cd, -(t.im * sd)), e * fma(t.im, cd, t.re * sd)};
}

// e^x for x <= 0 with the polynomial and table e2 of cexp_tab's modulus part, and ln 2
// subtracted in two parts (x spans the whole range of log-weight differences, and the
// result's relative error stays a few ulp throughout); x < -1000, and a NaN, give 0.
__device__ __forceinline__ double exp_tab(double x, const double *e2) {
  using namespace detail;
  constexpr double kRound = 0x1.8p52;
  x = fmax(x, -1000.0);
  const double kr = fma(x, 256.0 * kInvLn2, kRound);
  const int ki = __double2loint(kr);
  const double kx = kr - kRound;
  double r = fma(kx, -(kLn2Hi / 256.0), x);
  r = fma(kx, -(kLn2Lo / 256.0), r);
  double p = fma(r, kInvFact[4], kInvFact[3]);
  p = fma(p, r, kInvFact[2]);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p * e2[ki & 255], ki >> 8);
}

// exp(z) for the propagation factors in FP32, Re z <= 0 (Re z < -110 gives 0):
//   exp(x) = 2^k exp(r),  k = rint(x / ln 2),  r = x - k ln 2,  |r| <= ln(2)/2,
//   (cos y, sin y) = i^q (cos t, sin t),  q = rint(y 2/pi),  t = y - q pi/2,  |t| <= pi/4,
// with ln 2 and pi/2 split into two and three floats, and Taylor polynomials truncated
// after r^7 (exp), t^9 (sin) and t^10 (cos): remainders below 7e-9, 2e-9 and 2e-10.
__device__ __forceinline__ cplx<float> cexp(cplx<float> z) {
  constexpr float kInvLn2f = 0x1.715476p+0f, kLn2Hif = 0x1.62e430p-1f, kLn2Lof = -0x1.05c610p-29f;
  constexpr float kTwoOverPif = 0x1.45f306p-1f;
  constexpr float kPio2Af = 0x1.921fb6p+0f, kPio2Bf = -0x1.777a5cp-25f, kPio2Cf = -0x1.ee59dap-50f;
  const float x = z.re < -110.0f ? -110.0f : z.re;
  const float kx = rintf(x * kInvLn2f);
  float r = fmaf(kx, -kLn2Hif, x);
  r = fmaf(kx, -kLn2Lof, r);
  float p = 1.0f / 5040.0f;
  p = fmaf(p, r, 1.0f / 720.0f);
  p = fmaf(p, r, 1.0f / 120.0f);
  p = fmaf(p, r, 1.0f / 24.0f);
  p = fmaf(p, r, 1.0f / 6.0f);
  p = fmaf(p, r, 0.5f);
  p = fmaf(p, r, 1.0f);
  p = fmaf(p, r, 1.0f);
  const float e = ldexpf(p, (int)kx);

  const float qy = rintf(z.im * kTwoOverPif);
  float t = fmaf(qy, -kPio2Af, z.im);
  t = fmaf(qy, -kPio2Bf, t);
  t = fmaf(qy, -kPio2Cf, t);
  const float t2 = t * t;
  float S = 1.0f / 362880.0f;
  S = fmaf(S, t2, -1.0f / 5040.0f);
  S = fmaf(S, t2, 1.0f / 120.0f);
  S = fmaf(S, t2, -1.0f / 6.0f);
  const float st = fmaf(t * t2, S, t);
  float C = -1.0f / 3628800.0f;
  C = fmaf(C, t2, 1.0f / 40320.0f);
  C = fmaf(C, t2, -1.0f / 720.0f);
  C = fmaf(C, t2, 1.0f / 24.0f);
  C = fmaf(C, t2, -0.5f);
  const float ct = fmaf(t2, C, 1.0f);
  const int q = (int)qy;
  const float a = (q & 1) ? st : ct, b = (q & 1) ? ct : st;
  const float cy = ((q + 1) & 2) ? -a : a, sy = (q & 2) ? -b : b;
  return {e * cy, e * sy};
}

}  // namespace rjsmc
