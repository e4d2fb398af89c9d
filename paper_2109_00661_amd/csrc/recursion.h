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
// is carried in projective form: with R = A/B (A = k2_l - k2_{l+1}, B = (u_l+u_{l+1})^2)
// and r = N/D,
//   N_l = A D_{l+1} + B N_{l+1} E_{l+1},   D_l = B D_{l+1} + A N_{l+1} E_{l+1},
// so the whole stack needs one real division (Im r = Im(N conj D) / |D|^2) instead of
// two complex divisions per layer.  No lam - u or u_l - u_{l+1} is ever formed.
// FP64 keeps N, D unscaled (|D| stays within 1e-140 .. 1e30 for <= 16 layers of this
// system); FP32 rescales by a power of two every layer.
template <typename T>
__device__ __forceinline__ void rescale(cplx<T> &N, cplx<T> &D) {}
template <>
__device__ __forceinline__ void rescale<float>(cplx<float> &N, cplx<float> &D) {
  const float m = fabsf(D.re) + fabsf(D.im);
  const int e = -__builtin_amdgcn_frexp_expf(m);
  N = {ldexpf(N.re, e), ldexpf(N.im, e)};
  D = {ldexpf(D.re, e), ldexpf(D.im, e)};
}

// a b + c d with one multiplication and three fused multiply-adds per component.
template <typename T>
__device__ __forceinline__ cplx<T> cmul2add(cplx<T> a, cplx<T> b, cplx<T> c, cplx<T> d) {
  return {fma(a.re, b.re, fma(-a.im, b.im, fma(c.re, d.re, -(c.im * d.im)))),
          fma(a.re, b.im, fma(a.im, b.re, fma(c.re, d.im, c.im * d.re)))};
}

// Propagation factor exp(-2 h u): table-assisted in FP64, polynomial in FP32.
__device__ __forceinline__ cplx<double> prop_exp(cplx<double> z, const cplx<double> *phase,
                                                 const double *e2) {
  return cexp_tab(z, phase, e2);
}
__device__ __forceinline__ cplx<float> prop_exp(cplx<float> z, const cplx<double> *, const double *) {
  return cexp(z);
}

// Per-(frequency, layer) terms are read from LDS: k2[l] (layers 0..L-1), the interface
// numerators dk2[l] = k2[l] - k2[l+1] (l < L-1) and h2[l] = -2 h_l (l < L-1).  The layer
// loop is a runtime loop (unrolled by two, which removes the register rotation of the
// carried u and stays within 128 VGPRs) whose carried state is N, D and u_{l+1}.  phase / e2 are the
// LDS copies of the exponential's tables (used in FP64).
template <typename T>
__device__ __forceinline__ T reflection_im(T lam, const cplx<T> *k2, const cplx<T> *dk2, const T *h2, int L,
                                           const cplx<double> *phase, const double *e2) {
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
      const cplx<T> A = dk2[l];
      const cplx<T> B = csq(u + ub);
      const T hh = h2[l + 1];
      const cplx<T> NE = N * prop_exp(cplx<T>{hh * ub.re, hh * ub.im}, phase, e2);
      const cplx<T> Nn = cmul2add(A, D, B, NE);
      D = cmul2add(B, D, A, NE);
      N = Nn;
      rescale(N, D);
      ub = u;
    }
    const cplx<T> k0 = k2[0];
    const cplx<T> A0 = {-k0.re, -k0.im};
    const cplx<T> B0 = csq(cplx<T>{lam + ub.re, ub.im});
    const T hh = h2[0];
    const cplx<T> NE = N * prop_exp(cplx<T>{hh * ub.re, hh * ub.im}, phase, e2);
    const cplx<T> Nn = cmul2add(A0, D, B0, NE);
    D = cmul2add(B0, D, A0, NE);
    N = Nn;
  }
  return (N.im * D.re - N.re * D.im) * fast_rcp(D.re * D.re + D.im * D.im);
}

}  // namespace rjsmc
