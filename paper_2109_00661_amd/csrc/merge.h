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
// Decoupled layout: lane l loads conductivity row l and chargeability row l (interface
// and property) in one round of loads, and the ranks and segment counts are formed from
// those registers with wave shuffles, so a merge waits for two global loads in sequence
// (the counts, then everything else) whatever the layer counts.
// merge_counts takes the particle's counts (kappa, lambda; lambda is ignored for the
// merged layout) already loaded; merge_particle loads them.
__device__ __forceinline__ int merge_counts(const DevParticles &p, int64_t i, bool valid, int kap, int lam,
                                            int kc, int km, int lmax, LayerStack *st, int *flags) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t S = p.stride;
  const bool dec = p.layout == RJSMC_LAYOUT_DECOUPLED;
  int L = 0;
  bool ok = valid;
  if (!dec) lam = 0;
  if (ok) {
    L = kap + lam + 1;
    if (kap < 0 || lam < 0 || kap > kc || lam > (dec ? km : 0) || L > lmax) {
      if (lane == 0) atomicOr(flags, kFlagCapacity);
      ok = false;
    }
  }
  bool bad = false;
  if (ok && dec) {
    // lane l: conductivity row l (l < kap) and chargeability row l (l < lam)
    double zc = 0.0, ph = 0.0, zm = 0.0, mm = 0.0;
    if (lane < kap) {
      zc = p.z_cond[(int64_t)lane * S + i];
      ph = p.phi[(int64_t)lane * S + i];
    }
    if (lane < lam) {
      zm = p.z_charg[(int64_t)lane * S + i];
      mm = p.m[(int64_t)lane * S + i];
    }
    const double phib = p.phi_b[i];
    // this lane's interface in the merged order: conductivity row lane, or chargeability
    // row j = lane - kap; its rank counts the other partition's interfaces above it
    // (conductivity first on ties)
    const bool isc = lane < kap, ism = !isc && lane < kap + lam;
    const int j = ism ? lane - kap : 0;
    const double zmj = __shfl(zm, j);
    const double zmj1 = __shfl(zm, j > 0 ? j - 1 : 0);
    const double zc1 = __shfl(zc, lane > 0 ? lane - 1 : 0);
    const double z = isc ? zc : zmj;
    int rank = isc ? lane : j;
    // (every lane takes part in each shuffle: a shuffle under a lane condition would
    // read lanes that are not active there)
    for (int t = 0; t < lam; ++t) {
      const double y = __shfl(zm, t);
      rank += (isc && y < z) ? 1 : 0;
    }
    for (int t = 0; t < kap; ++t) {
      const double y = __shfl(zc, t);
      rank += (ism && y <= z) ? 1 : 0;
    }
    if (isc && lane > 0 && !(z >= zc1)) bad = true;
    if (ism && j > 0 && !(z >= zmj1)) bad = true;
    if ((isc || ism) && !(z >= 0.0)) bad = true;
    if (isc || ism) {
      st->top[rank + 1] = z;
      st->src_top[rank + 1] = isc ? lane : kMaxLayers + j;
    }
    if (lane == 0) {
      st->top[0] = 0.0;
      st->src_top[0] = -1;
    }
    const bool any_bad = __any(bad);
    wave_lds_sync();
    if (any_bad) {
      if (lane == 0) atomicOr(flags, kFlagUnsorted);
      ok = false;
    } else {
      // layer `lane`: the segments of each partition above its top
      const double top = lane < L ? st->top[lane] : 0.0;
      int ic = 0, im = 0;
      for (int t = 0; t < kap; ++t) ic += __shfl(zc, t) <= top ? 1 : 0;
      for (int t = 0; t < lam; ++t) im += __shfl(zm, t) <= top ? 1 : 0;
      const double phs = __shfl(ph, ic > 0 ? ic - 1 : 0);
      const double ms = __shfl(mm, im > 0 ? im - 1 : 0);
      if (lane < L) {
        const double phi = ic == 0 ? phib : phs;
        st->sig[lane] = exp(phi * 2.302585092994045684);
        st->src_sig[lane] = ic - 1;
        st->m[lane] = im == 0 ? 0.0 : ms;
        st->src_m[lane] = im - 1;
      }
    }
  } else if (ok) {
    if (lane < kap) {
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
    const bool any_bad = __any(bad);
    wave_lds_sync();
    if (any_bad) {
      if (lane == 0) atomicOr(flags, kFlagUnsorted);
      ok = false;
    } else if (lane < L) {
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

__device__ __forceinline__ int merge_particle(const DevParticles &p, int64_t i, bool valid, int kc,
                                              int km, int lmax, LayerStack *st, int *flags) {
  int kap = 0, lam = 0;
  if (valid) {
    kap = p.kappa[i];
    lam = p.layout == RJSMC_LAYOUT_DECOUPLED ? p.lambda[i] : 0;
  }
  return merge_counts(p, i, valid, kap, lam, kc, km, lmax, st, flags);
}

}  // namespace rjsmc
