// Projective form of the layered-earth TE reflection recursion (shared by the forward
// and adjoint kernels).
#pragma once

#include "cplx.h"

namespace rjsmc {

// Imaginary part of the TE reflection coefficient at the surface for wavenumber lam,
// layer wavenumbers k2[l] = i w mu0 sigma_hat_l and thicknesses thk[l] (layers
// 0..L-1, the last one infinite).  The generalized reflection recursion
//   R_{l,l+1} = (k2_l - k2_{l+1}) / (u_l + u_{l+1})^2,   R_air = -k2_0 / (lam + u_0)^2,
//   r_l = (R_{l,l+1} + r_{l+1} E_{l+1}) / (1 + R_{l,l+1} r_{l+1} E_{l+1}),
//   E_l = exp(-2 u_l h_l),  u_l = sqrt(lam^2 + k2_l), Re u_l > 0,
// is carried in projective form, r = N/D: the deepest interface starts from
// N = k2_{L-2} - k2_{L-1}, D = (u_{L-2} + u_{L-1})^2 (R without a difference of nearly
// equal u), and every interface above takes one projective step, so the whole stack
// needs one real division (Im r = Im(N conj D) / |D|^2) instead of two complex
// divisions per layer.  FP64 takes step_up (two complex products; it forms u_l -
// u_{l+1} implicitly, which costs FP64 nothing measurable); FP32 takes step_ratio,
// whose interface numerator is the difference of the layer wavenumbers k2_l -
// k2_{l+1} (exact for equal layers, no cancellation of nearly equal u).  FP64 keeps
// N, D unscaled (each step multiplies them by about |u|, so |D| stays far inside the
// FP64 range for <= 16 layers of this system); FP32 rescales by a power of two every
// layer.
template <typename T>
__device__ __forceinline__ void rescale(cplx<T> &N, cplx<T> &D) {}
template <>
__device__ __forceinline__ void rescale<float>(cplx<float> &N, cplx<float> &D) {
  const float m = fabsf(D.re) + fabsf(D.im);
  const int e = -__builtin_amdgcn_frexp_expf(m);
  N = {ldexpf(N.re, e), ldexpf(N.im, e)};
  D = {ldexpf(D.re, e), ldexpf(D.im, e)};
}

// One interface upwards in projective form, with a = u above and b = u below it:
// R = (a - b) / (a + b), and r_above = (R + r E) / (1 + R r E) for r = N / D becomes
//   N' = a S - b T,  D' = a S + b T,  S = D + N E,  T = D - N E
// (the common factor a + b dropped): two complex products instead of four, and neither
// the interface numerator nor (a + b)^2 is formed.  a - b never appears explicitly: for
// nearly equal a and b (|k2| << lam^2, low frequencies and large lam) the D-part of N'
// is the difference of a S and b T, accurate only to a rounding of |a D| absolute.  In
// FP64 that is ~1e-16 of r; in FP32 it would be 6e-8 |a D|, which for k2 / lam^2 ~ 1e-5
// is a relative error of ~1e-2 in N', so FP32 uses step_ratio instead.
template <typename T>
__device__ __forceinline__ void step_up(cplx<T> &N, cplx<T> &D, cplx<T> a, cplx<T> b, cplx<T> E) {
  const cplx<T> NE = N * E;
  const cplx<T> S = D + NE, Tm = D - NE;
  const cplx<T> P = a * S, Q = b * Tm;
  N = P - Q;
  D = P + Q;
}
// The same step at the air interface, where a = lam is real (two products fewer: a zero
// imaginary part would still be multiplied out, since 0 x is not folded without
// fast-math; the results are the same).
template <typename T>
__device__ __forceinline__ void step_up(cplx<T> &N, cplx<T> &D, T a, cplx<T> b, cplx<T> E) {
  const cplx<T> NE = N * E;
  const cplx<T> S = D + NE, Tm = D - NE;
  const cplx<T> P = a * S, Q = b * Tm;
  N = P - Q;
  D = P + Q;
}

// The same step with R = dk / B, dk = a^2 - b^2 = k2_above - k2_below (lam^2 cancels
// exactly) and B = (a + b)^2:
//   N' = dk D + B N E,  D' = B D + dk N E
// (the common factor 1 / B dropped).  Every factor is formed without subtracting
// nearly equal numbers, so each step is accurate to a few roundings relative to its
// terms whatever the ratio k2 / lam^2.
template <typename T>
__device__ __forceinline__ void step_ratio(cplx<T> &N, cplx<T> &D, cplx<T> dk, cplx<T> B, cplx<T> E) {
  const cplx<T> NE = N * E;
  const cplx<T> Np = dk * D + B * NE;
  D = B * D + dk * NE;
  N = Np;
}

// Propagation factor exp(-2 h u): table-assisted in FP64, polynomial in FP32.
__device__ __forceinline__ cplx<double> prop_exp(cplx<double> z, const cplx<double> *phase,
                                                 const double *e2, ExpConsts kc) {
  return cexp_tab(z, phase, e2, kc);
}
__device__ __forceinline__ cplx<float> prop_exp(cplx<float> z, const cplx<double> *, const double *, ExpConsts) {
  return cexp(z);
}

// Per-(frequency, layer) terms are read from LDS: k2[l] (layers 0..L-1), the interface
// numerators dk2[l] = k2[l] - k2[l+1] (l < L-1) and h2[l] = -2 h_l (l < L-1).  The layer
// loop is a runtime loop (unrolled by two, which removes the register rotation of the
// carried u and stays within 128 VGPRs) whose carried state is N, D and u_{l+1}.  phase / e2 are the
// LDS copies of the exponential's tables and kc its polynomial constants from exp_consts()
// (used in FP64).
template <typename T>
__device__ __forceinline__ T reflection_im(T lam, const cplx<T> *k2, const cplx<T> *dk2, const T *h2, int L,
                                           const cplx<double> *phase, const double *e2, ExpConsts kc) {
  constexpr bool kRatio = sizeof(T) == sizeof(float);   // FP32: cancellation-free steps
  const T lam2 = lam * lam;
  const cplx<T> kb = k2[L - 1];
  cplx<T> ub = csqrt_fast(cplx<T>{lam2 + kb.re, kb.im});
  cplx<T> N, D;
  if (L == 1) {
    N = {-kb.re, -kb.im};
    D = csq(cplx<T>{lam + ub.re, ub.im});
  } else {
    {
      const cplx<T> kl = k2[L - 2];
      const cplx<T> u = csqrt_fast(cplx<T>{lam2 + kl.re, kl.im});
      N = dk2[L - 2];
      D = csq(u + ub);
      ub = u;
    }
#pragma unroll 2
    for (int l = L - 3; l >= 0; --l) {
      const cplx<T> kl = k2[l];
      const cplx<T> u = csqrt_fast(cplx<T>{lam2 + kl.re, kl.im});
      const T hh = h2[l + 1];
      const cplx<T> E = prop_exp(cplx<T>{hh * ub.re, hh * ub.im}, phase, e2, kc);
      if (kRatio)
        step_ratio(N, D, dk2[l], csq(u + ub), E);
      else
        step_up(N, D, u, ub, E);
      rescale(N, D);
      ub = u;
    }
    const T hh = h2[0];
    const cplx<T> E0 = prop_exp(cplx<T>{hh * ub.re, hh * ub.im}, phase, e2, kc);
    if (kRatio)   // air interface: lam^2 - u_0^2 = -k2_0
      step_ratio(N, D, cplx<T>{-k2[0].re, -k2[0].im}, csq(cplx<T>{lam + ub.re, ub.im}), E0);
    else
      step_up(N, D, lam, ub, E0);
  }
  return (N.im * D.re - N.re * D.im) * fast_rcp(D.re * D.re + D.im * D.im);
}

}  // namespace rjsmc
