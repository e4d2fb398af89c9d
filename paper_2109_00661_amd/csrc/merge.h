// Per-particle merge of the decoupled conductivity and chargeability partitions into one
// layer stack (paper Section 2.1, Fig. 2: the two change-point profiles are combined by
// a direct sum).  One wavefront works on one particle; the result lands in LDS.
#pragma once

#include "rjsmc_internal.h"

namespace rjsmc {

// Layer stack of one particle in LDS.  top[l] is the depth of the top of layer l
// (top[0] = 0); layer l has thickness top[l+1] - top[l]; the last layer is the
// basement.  src_* record which parameter each layer property and interface came from
// (used by the adjoint to route derivatives back):
//   src_sig[l]  = -1 for phi_b, else the row of phi
//   src_m[l]    = -1 for the zero-chargeability top segment, else the row of m
//   src_top[l]  = interface feeding top[l] (l >= 1): row of z_cond, or
//                 kMaxLayers + row of z_charg
struct LayerStack {
  double top[kMaxLayers + 1];
  double sig[kMaxLayers];     // sigma_inf (S/m)
  double m[kMaxLayers];       // chargeability
  int src_sig[kMaxLayers];
  int src_m[kMaxLayers];
  int src_top[kMaxLayers + 1];
  int L;                      // number of layers, 0 if the particle is invalid
};

// Lanes of one wavefront cooperate; `st` is this wave's LDS slot.  All 64 lanes of the
// wave must call this (it syncs the wave twice); a wave without a particle passes
// valid = false.  Returns L (>= 1) or 0 for no / an invalid particle (flags raised).
// Property rule: a layer takes the conductivity segment below the last conductivity
// interface at or above its top, and likewise for chargeability (zero above the first
// chargeability interface).
__device__ __forceinline__ int merge_particle(const DevParticles &p, int64_t i, bool valid, int kc,
                                              int km, int lmax, LayerStack *st, int *flags) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t S = p.stride;
  const bool dec = p.layout == RJSMC_LAYOUT_DECOUPLED;
  int kap = 0, lam = 0, L = 0;
  bool ok = valid;
  if (ok) {
    kap = p.kappa[i];
    lam = dec ? p.lambda[i] : 0;
    L = kap + lam + 1;
    if (kap < 0 || lam < 0 || kap > kc || lam > (dec ? km : 0) || L > lmax) {
      if (lane == 0) atomicOr(flags, kFlagCapacity);
      ok = false;
    }
  }
  bool bad = false;
  if (ok) {
    if (dec) {
      // rank of each interface in the merged order (conductivity first on ties)
      if (lane < kap + lam) {
        double z;
        int rank, src;
        if (lane < kap) {
          z = p.z_cond[(int64_t)lane * S + i];
          rank = lane;
          for (int j = 0; j < lam; ++j) rank += p.z_charg[(int64_t)j * S + i] < z;
          src = lane;
          if (lane > 0 && !(z >= p.z_cond[(int64_t)(lane - 1) * S + i])) bad = true;
        } else {
          const int j = lane - kap;
          z = p.z_charg[(int64_t)j * S + i];
          rank = j;
          for (int t = 0; t < kap; ++t) rank += p.z_cond[(int64_t)t * S + i] <= z;
          src = kMaxLayers + j;
          if (j > 0 && !(z >= p.z_charg[(int64_t)(j - 1) * S + i])) bad = true;
        }
        if (!(z >= 0.0)) bad = true;
        st->top[rank + 1] = z;
        st->src_top[rank + 1] = src;
      }
    } else if (lane < kap) {
      const double z = p.z_cond[(int64_t)lane * S + i];
      if (lane > 0 && !(z >= p.z_cond[(int64_t)(lane - 1) * S + i])) bad = true;
      if (!(z >= 0.0)) bad = true;
      st->top[lane + 1] = z;
      st->src_top[lane + 1] = lane;
    }
    if (lane == 0) {
      st->top[0] = 0.0;
      st->src_top[0] = -1;
    }
  }
  const bool any_bad = __any(bad);
  wave_lds_sync();
  if (ok && any_bad) {
    if (lane == 0) atomicOr(flags, kFlagUnsorted);
    ok = false;
  }
  if (ok && lane < L) {
    const double top = st->top[lane];
    if (dec) {
      int ic = 0, im = 0;
      for (int t = 0; t < kap; ++t) ic += p.z_cond[(int64_t)t * S + i] <= top;
      for (int j = 0; j < lam; ++j) im += p.z_charg[(int64_t)j * S + i] <= top;
      const double phi = ic == 0 ? p.phi_b[i] : p.phi[(int64_t)(ic - 1) * S + i];
      st->sig[lane] = exp(phi * 2.302585092994045684);
      st->src_sig[lane] = ic - 1;
      st->m[lane] = im == 0 ? 0.0 : p.m[(int64_t)(im - 1) * S + i];
      st->src_m[lane] = im - 1;
    } else {
      const double phi = lane == 0 ? p.phi_b[i] : p.phi[(int64_t)(lane - 1) * S + i];
      st->sig[lane] = exp(phi * 2.302585092994045684);
      st->src_sig[lane] = lane - 1;
      st->m[lane] = p.m[(int64_t)lane * S + i];
      st->src_m[lane] = lane;
    }
  }
  if (ok && lane == 0) st->L = L;
  wave_lds_sync();
  return ok ? L : 0;
}

}  // namespace rjsmc
