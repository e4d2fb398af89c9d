// Fused forward model + Gaussian log-likelihood for gfx950.
//
// One wavefront evaluates one particle.  Its 64 lanes tile the (frequency, filter
// abscissa) plane as 8 frequency groups x 8 abscissa groups: lane (g_w, g_l) handles
// frequencies g_w + 8q and abscissae g_l + 8s, so 40 x 120 pairs give exactly 75 per
// lane and the layer loop is uniform across the wave (one particle, one layer count).
// Per pair the lane runs the TE reflection recursion in registers (a runtime layer
// loop over LDS-resident k^2 and thicknesses); partial Hankel sums of Im r_TE are reduced over the
// 8 abscissa groups with xor shuffles, the 40 values go through LDS, and 20 lanes apply
// the frequency-to-time matrix and the likelihood terms.  After the workgroup stages the
// shared tables in LDS its waves run independently (wave-level syncs only), so a
// particle with few layers does not wait for a deeper neighbour.  The kernel is bound
// by FP64 (or FP32) vector ALU work: ~24,000 layer steps per particle for 5 layers.
// Small populations can take the spread evaluation instead (spread_terms_kernel and
// spread_finish_kernel below): the reflection terms of all particles dealt over every
// compute unit in ranges of equal work, then summed in the same order.
#include <hip/hip_runtime.h>

#include "cplx.h"
#include "merge.h"
#include "recursion.h"
#include "rjsmc_internal.h"

namespace rjsmc {

constexpr double kMu0 = 1.25663706143591729539e-06;   // 4 pi 1e-7
constexpr double kTwoPi = 6.28318530717958647692;

template <typename T>
__device__ __forceinline__ T to(double x) {
  return static_cast<T>(x);
}

// Per-particle Cole-Cole constants: (i w tau)^c = (w tau)^c (cos(pi c/2) + i sin(pi c/2)).
struct ColeCole {
  double c, log_tau, spc, cpc;
};
__device__ __forceinline__ ColeCole cole_cole(const DevParticles &p, int64_t i) {
  ColeCole cc;
  cc.c = p.c[i];
  cc.log_tau = p.log10_tau[i] * 2.302585092994045684;
  sincospi(0.5 * cc.c, &cc.spc, &cc.cpc);
  return cc;
}

// h2[l] = -2 h_l for the L - 1 finite layers (lane l).
template <typename T>
__device__ __forceinline__ void stage_h2(const LayerStack *st, int L, T *h2, int lane) {
  if (lane < L - 1) h2[lane] = T(-2) * to<T>(st->top[lane + 1] - st->top[lane]);
}

// Layer wavenumbers of one particle at angular frequency w (logw = log w, from the
// workgroup's table): k2[l] = i w mu0 sigma_inf_l (1 - m_l q_cc) with q_cc = 1 / (1 +
// (i w tau)^c), and the interface numerators dk2[l] = k2[l] - k2[l+1].  k2_freq holds the
// per-frequency factors, k2_layer forms one layer's value from them; every kernel builds
// its tables from these two, so the values are the same bits whoever forms them.
template <typename T>
struct K2Freq {
  T wmu;
  cplx<T> qt;
};
template <typename T>
__device__ __forceinline__ K2Freq<T> k2_freq(double w, double logw, const ColeCole &cc) {
  const double wtc = exp(cc.c * (logw + cc.log_tau));
  const cplx<double> qcc = crcp(cplx<double>{1.0 + wtc * cc.cpc, wtc * cc.spc});
  return K2Freq<T>{to<T>(w * kMu0), cplx<T>{to<T>(qcc.re), to<T>(qcc.im)}};
}
template <typename T>
__device__ __forceinline__ cplx<T> k2_layer(const LayerStack *st, int l, const K2Freq<T> &kf) {
  const T sg = to<T>(st->sig[l]), mg = to<T>(st->m[l]);
  const cplx<T> sh = {sg * (T(1) - mg * kf.qt.re), sg * (-(mg * kf.qt.im))};
  return cplx<T>{-(kf.wmu * sh.im), kf.wmu * sh.re};
}

// The table of one frequency, by the 8 lanes gl of a frequency group (layers gl, gl + 8).
template <typename T>
__device__ __forceinline__ void stage_k2(const LayerStack *st, int L, double w, double logw, const ColeCole &cc,
                                         int gl, cplx<T> *k2, cplx<T> *dk2) {
  const K2Freq<T> kf = k2_freq<T>(w, logw, cc);
  for (int l = gl; l < L; l += 8) {
    const cplx<T> kl = k2_layer<T>(st, l, kf);
    k2[l] = kl;
    if (l + 1 < L) dk2[l] = kl - k2_layer<T>(st, l + 1, kf);
  }
}

// Gate responses of particle i from its Im H values (imh[0..n_freq), LDS) and its
// log-likelihood, by one whole wave: lane g < n_gate forms gate g, the wave adds the
// likelihood terms.
__device__ __forceinline__ void gates_loglik(const DevSystem &s, const DevParticles &p, int64_t i, const double *K,
                                             const double *imh, const double *eps2, double *resp,
                                             const double *y_obs, double *ll, int lane) {
  const int nf = s.n_freq, ng = s.n_gate;
  double term = 0.0;
  if (lane < ng) {
    double y = 0.0;
    for (int j = 0; j < nf; ++j) y += K[lane * nf + j] * imh[j];
    if (resp) resp[i * ng + lane] = y;
    if (ll) {
      const int64_t snd = p.n_per_sounding > 0 ? i / p.n_per_sounding : 0;
      const double d = y_obs[snd * ng + lane];
      const double e = s.eps_mn * y;
      const double s2 = eps2[lane] + e * e;
      const double r = d - y;
      term = r * r / s2 + log(kTwoPi * s2);
    }
  }
  if (ll) {
    term += __shfl_xor(term, 1);
    term += __shfl_xor(term, 2);
    term += __shfl_xor(term, 4);
    term += __shfl_xor(term, 8);
    term += __shfl_xor(term, 16);
    term += __shfl_xor(term, 32);
    if (lane == 0) {
      const double v = -0.5 * term;
      ll[i] = (v == v && v != HUGE_VAL) ? v : -HUGE_VAL;   // NaN or +inf -> -inf
    }
  }
}

// An invalid particle: NaN responses, -inf log-likelihood.
__device__ __forceinline__ void invalid_outputs(const DevSystem &s, int64_t i, double *resp, double *ll, int lane) {
  if (resp && lane < s.n_gate) resp[i * s.n_gate + lane] = __builtin_nan("");
  if (ll && lane == 0) ll[i] = -HUGE_VAL;
}

// resp != nullptr: write gate responses.  ll != nullptr: write the log-likelihood.
// WPB particles per workgroup, P waves per particle: wave q0 of a particle takes the
// frequency groups q0, q0 + P, ... (P = 1: the whole particle; P > 1 shortens the
// latency of small batches), and the particle's first wave applies the gates and the
// likelihood after a workgroup barrier.  perm != nullptr: slot j of the grid evaluates
// particle perm[j] (workgroups in launch order, dealt round-robin to the XCDs);
// otherwise slot j is particle j (workgroups renumbered XCD-contiguous).
template <typename T, int WPB, int P>
__global__ __launch_bounds__(kWave * WPB * P, 16 / (WPB * P) > 0 ? 16 / (WPB * P) : 1) void forward_kernel(
    DevSystem s, DevParticles p, int kc, int km, double *resp, const double *y_obs, double *ll,
    const int32_t *perm) {
  constexpr int LMAX = kMaxLayers;
  constexpr int kWavesPerBlock = WPB * P;
  __shared__ double s_lam[kMaxHankel];
  __shared__ double s_ck[kMaxHankel];
  __shared__ double s_omega[kMaxFreq];
  __shared__ double s_logw[kMaxFreq];
  __shared__ double s_eps2[kMaxGate];
  __shared__ cplx<double> s_phase[kPhaseN];
  __shared__ double s_exp2[kExp2N];
  __shared__ LayerStack s_stack[kWavesPerBlock];
  __shared__ double s_imh[WPB][kMaxFreq];
  __shared__ cplx<T> s_k2[kWavesPerBlock][8][LMAX];
  __shared__ cplx<T> s_dk2[kWavesPerBlock][8][LMAX];
  __shared__ T s_h2[kWavesPerBlock][LMAX];
  extern __shared__ double s_K[];   // [n_gate][n_freq], dynamic

  const int nf = s.n_freq, ng = s.n_gate, nhp = s.n_hankel_pad;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int pw = wave / P;           // particle of this wave within the workgroup
  const int q0 = wave % P;           // first frequency group of this wave
  const int64_t slot = (int64_t)(perm ? blockIdx.x : xcd_block(blockIdx.x, gridDim.x)) * WPB + pw;
  const int64_t i = perm ? (slot < p.n ? (int64_t)perm[slot] : p.n) : slot;
  const bool valid = i < p.n;
  const bool skip = valid && p.mask && p.mask[i] != p.mask_value;
  // workgroups with no particle to evaluate (masked launches) leave before staging
  if (!__syncthreads_or(valid && !skip)) return;
  for (int t = threadIdx.x; t < nhp; t += blockDim.x) {
    s_lam[t] = s.lam[t];
    s_ck[t] = s.ck[t];
  }
  for (int t = threadIdx.x; t < nf; t += blockDim.x) {
    s_omega[t] = s.omega[t];
    s_logw[t] = log(s.omega[t]);
  }
  for (int t = threadIdx.x; t < nf * ng; t += blockDim.x) s_K[t] = s.K[t];
  for (int t = threadIdx.x; t < ng; t += blockDim.x) s_eps2[t] = s.eps_an2[t];
  for (int t = threadIdx.x; t < kPhaseN; t += blockDim.x)
    s_phase[t] = cplx<double>{s.phase[2 * t], s.phase[2 * t + 1]};
  for (int t = threadIdx.x; t < kExp2N; t += blockDim.x) s_exp2[t] = s.exp2t[t];
  LayerStack *st = &s_stack[wave];
  __syncthreads();
  // the wave's particle is one, so its merged-layer count is wave-uniform: held in a
  // scalar register, the layer loops count in scalar instructions
  const int L = __builtin_amdgcn_readfirstlane(merge_particle(p, i, valid && !skip, kc, km, LMAX, st, s.flags));

  ColeCole cc{0.0, 0.0, 0.0, 1.0};
  if (L > 0) {
    cc = cole_cole(p, i);
    stage_h2<T>(st, L, s_h2[wave], lane);
  }
  const int gl = lane & 7, gw = lane >> 3;
  const int nhg = nhp >> 3;
  const int nq = (nf + 7) >> 3;
  const ExpConsts ek = exp_consts();
  // With more waves per particle than frequency chunks, each chunk's abscissa groups are
  // split into A parts (work unit = chunk x part); the parts store their reflection
  // terms and the particle's first wave adds them in the order of the A == 1 path, so
  // every tile shape gives the same sums.
  const int A = (P > 1 && P > nq) ? P / nq : 1;
  double *s_rim = s_K + nf * ng + pw * nf * nhp;   // [nf][nhp] reflection terms when A > 1
  // the waves of a workgroup run independently from here on (wave-level syncs only)
#pragma unroll 1
  for (int u = q0; u < nq * A; u += P) {
    const int q = A == 1 ? u : u / A, part = u - q * A;
    const int jf = gw + 8 * q;
    const bool act = L > 0 && jf < nf;
    if (act) stage_k2<T>(st, L, s_omega[jf], s_logw[jf], cc, gl, s_k2[wave][gw], s_dk2[wave][gw]);
    wave_lds_sync();
    if (act && A == 1) {
      double acc = 0.0;
#pragma unroll 1
      for (int sidx = 0; sidx < nhg; ++sidx) {
        const int k = gl + 8 * sidx;
        const T rim = reflection_im<T>(to<T>(s_lam[k]), s_k2[wave][gw], s_dk2[wave][gw], s_h2[wave], L,
                                         s_phase, s_exp2, ek);
        acc = __builtin_fma(s_ck[k], static_cast<double>(rim), acc);
      }
      // reduce over the 8 abscissa groups (lane bits 0..2); all 8 lanes of a group
      // share jf, so a group is either wholly active or wholly idle here
      acc += __shfl_xor(acc, 1);
      acc += __shfl_xor(acc, 2);
      acc += __shfl_xor(acc, 4);
      if (gl == 0) s_imh[pw][jf] = acc;
    } else if (act) {
#pragma unroll 1
      for (int sidx = part * nhg / A; sidx < (part + 1) * nhg / A; ++sidx) {
        const int k = gl + 8 * sidx;
        s_rim[jf * nhp + k] = static_cast<double>(reflection_im<T>(to<T>(s_lam[k]), s_k2[wave][gw],
                                                                   s_dk2[wave][gw], s_h2[wave], L, s_phase,
                                                                   s_exp2, ek));
      }
    }
    wave_lds_sync();
  }
  if (P > 1) {
    __syncthreads();                 // every wave of the particle has written its terms or Im H
    if (q0 != 0) return;
  }
  if (A > 1 && L > 0) {
    // Im H from the stored terms, added in the order of the A == 1 path
    for (int qq = 0; qq < nq; ++qq) {
      const int jf = gw + 8 * qq;
      double acc = 0.0;
      if (jf < nf)
        for (int sidx = 0; sidx < nhg; ++sidx) {
          const int k = gl + 8 * sidx;
          acc = __builtin_fma(s_ck[k], s_rim[jf * nhp + k], acc);
        }
      acc += __shfl_xor(acc, 1);
      acc += __shfl_xor(acc, 2);
      acc += __shfl_xor(acc, 4);
      if (gl == 0 && jf < nf) s_imh[pw][jf] = acc;
    }
    wave_lds_sync();
  }
  if (L > 0)
    gates_loglik(s, p, i, s_K, s_imh[pw], s_eps2, resp, y_obs, ll, lane);
  else if (valid && !skip)
    invalid_outputs(s, i, resp, ll, lane);
}

// ---- spread evaluation (FP64): a launch's work dealt evenly over the compute units
// With one particle per workgroup a small population ends when its deepest particle does,
// on one compute unit.  Here a particle's reflection terms are cut into units (frequency
// chunk q, abscissa step s: the 64 terms of frequencies gw + 8q at abscissae gl + 8s, one
// per lane); unit j = q n_hg + s of the particle in slot r weighs its layer capacity + 1,
// and the units, slot-major, are cut into ranges of equal weight, one per workgroup of a
// grid with one workgroup per compute unit.  A deep particle's units so spread over more
// compute units than a shallow one's.  A workgroup merges the few particles of its range
// (as many as fit a pool of kSpreadPool layer tables, at most kSpreadStage at a time) and
// builds their wavenumber tables in LDS together; then its waves claim the range's units
// one at a time from an LDS counter, so that every SIMD stays busy until the range is
// done.  spread_terms_kernel writes the terms to rim in
// [slot][q][s][lane] order; spread_finish_kernel adds them in the order of forward_kernel
// and applies the gates and the likelihood, so the results are the same bits.
constexpr int kSpreadWaves = 16;                         // waves per workgroup
constexpr int kSpreadMaxN = 2 * kWave * kSpreadWaves;   // particles per launch (two per thread)
constexpr int kSpreadStage = 8;                          // particles staged at once, at most
constexpr int kSpreadPool = 64;                          // layer capacities staged at once, at most

// Weight of the particle in a slot: 0 if masked out, else its layer capacity (clamped to
// 1..kMaxLayers, so that invalid counts stay bounded) + 1.  Its counts are kept for the
// merge.
__device__ __forceinline__ int spread_weight(const DevParticles &p, int64_t i, int *kap, int *lam) {
  *kap = p.kappa[i];
  *lam = p.layout == RJSMC_LAYOUT_DECOUPLED ? p.lambda[i] : 0;
  if (p.mask && p.mask[i] != p.mask_value) return 0;
  int cap = *kap + *lam + 1;
  cap = cap < 1 ? 1 : (cap > kMaxLayers ? kMaxLayers : cap);
  return cap + 1;
}

// Dynamic LDS of spread_terms_kernel: the staged particles' k2 and dk2 tables, each
// particle's [n_freq][capacity] behind the previous one's.
template <typename T>
static size_t spread_table_bytes(const DevSystem &s) {
  return 2 * sizeof(cplx<T>) * kSpreadPool * s.n_freq;
}

// rim_layers[r] = L of the particle in slot r (0: invalid), written by the workgroup that
// holds the slot's first unit (masked slots are not written).
template <typename T>
__global__ __launch_bounds__(kWave * kSpreadWaves, 1) void spread_terms_kernel(
    DevSystem s, DevParticles p, int kc, int km, const int32_t *perm, double *rim, int32_t *rim_layers) {
  constexpr int LMAX = kMaxLayers;
  constexpr int KP = kSpreadStage;
  static_assert(kSpreadPool >= kMaxLayers, "one particle of any capacity fits the pool");
  __shared__ double s_lam[kMaxHankel];
  __shared__ double s_omega[kMaxFreq];
  __shared__ double s_logw[kMaxFreq];
  __shared__ cplx<double> s_phase[kPhaseN];
  __shared__ double s_exp2[kExp2N];
  __shared__ int s_pref[kSpreadMaxN + 1];   // s_pref[r] = weight of slots 0..r-1
  __shared__ int s_kap[kSpreadMaxN], s_lmb[kSpreadMaxN];   // counts of slot r
  __shared__ int s_wsum[kSpreadWaves];
  __shared__ LayerStack s_stack[KP];
  __shared__ ColeCole s_cc[KP];
  __shared__ T s_h2[KP][LMAX];
  __shared__ int s_L[KP];
  // staged set: slot, first unit, first claim (entry np: the claims in all), table offset
  // and capacity
  __shared__ int s_sl[KP], s_ja[KP], s_cu[KP + 1], s_off[KP], s_cap[KP], s_np;
  __shared__ int s_next;
  extern __shared__ double s_tab[];   // k2 pool [kSpreadPool n_freq], then dk2 alike
  const int nf = s.n_freq, nhp = s.n_hankel_pad;
  cplx<T> *const s_k2 = reinterpret_cast<cplx<T> *>(s_tab);
  cplx<T> *const s_dk2 = s_k2 + kSpreadPool * nf;

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x & (kWave - 1);
  const int n = (int)p.n;   // 1..kSpreadMaxN (the host checks)
  for (int t = threadIdx.x; t < nhp; t += blockDim.x) s_lam[t] = s.lam[t];
  for (int t = threadIdx.x; t < nf; t += blockDim.x) {
    s_omega[t] = s.omega[t];
    s_logw[t] = log(s.omega[t]);
  }
  for (int t = threadIdx.x; t < kPhaseN; t += blockDim.x)
    s_phase[t] = cplx<double>{s.phase[2 * t], s.phase[2 * t + 1]};
  for (int t = threadIdx.x; t < kExp2N; t += blockDim.x) s_exp2[t] = s.exp2t[t];
  if (threadIdx.x == 0) s_next = 0;
  // prefix sums of the slot weights: thread t holds slots 2t and 2t + 1
  const int r0 = 2 * (int)threadIdx.x;
  int k0 = 0, l0 = 0, k1 = 0, l1 = 0;
  const int w0 = r0 < n ? spread_weight(p, perm ? (int64_t)perm[r0] : r0, &k0, &l0) : 0;
  const int w1 = r0 + 1 < n ? spread_weight(p, perm ? (int64_t)perm[r0 + 1] : r0 + 1, &k1, &l1) : 0;
  int x = w0 + w1;
  for (int d = 1; d < kWave; d <<= 1) {
    const int y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == kWave - 1) s_wsum[wave] = x;
  if (r0 < n) {
    s_kap[r0] = k0;
    s_lmb[r0] = l0;
  }
  if (r0 + 1 < n) {
    s_kap[r0 + 1] = k1;
    s_lmb[r0 + 1] = l1;
  }
  __syncthreads();
  for (int v = 0; v < wave; ++v) x += s_wsum[v];
  if (r0 < n) s_pref[r0 + 1] = x - w1;
  if (r0 + 1 < n) s_pref[r0 + 2] = x;
  if (threadIdx.x == 0) s_pref[0] = 0;
  __syncthreads();

  // this workgroup's range: the units whose weight offset lies in [lo, hi).  Every wave
  // derives the same bounds and staged sets; readfirstlane keeps the values it reads from
  // LDS in scalar registers.
  auto uni = [](int v) { return __builtin_amdgcn_readfirstlane(v); };
  const int nq = (nf + 7) >> 3, nhg = nhp >> 3, U = nq * nhg;
  const int64_t total = (int64_t)U * uni(s_pref[n]);
  const int64_t G = gridDim.x;
  const int64_t lo = ((int64_t)blockIdx.x * total + G - 1) / G;
  const int64_t hi = (((int64_t)blockIdx.x + 1) * total + G - 1) / G;
  if (lo >= hi) return;   // workgroup-uniform: an empty range
  // The slot holding offset x: the first r with U s_pref[r + 1] > x (its weight is > 0),
  // by a 64-way search in two rounds (n <= 64 x 32): the first segment of 32 slots whose
  // last slot qualifies, then the first qualifying slot in it (slots beyond n - 1 test
  // slot n - 1, which qualifies for x < total).
  auto slot_of = [&](int64_t x) {
    const int c1 = min(32 * lane + 31, n - 1);
    const uint64_t m1 = __ballot((int64_t)U * s_pref[c1 + 1] > x);
    const int seg = 32 * __builtin_ctzll(m1);
    const int c2 = min(seg + (lane & 31), n - 1);
    const uint64_t m2 = __ballot((int64_t)U * s_pref[c2 + 1] > x);
    return uni(seg + __builtin_ctzll(m2));
  };
  // first slot and its first unit in the range; last slot and its units below hi
  const int r_first = slot_of(lo), r_last = slot_of(hi - 1);
  int j_first, j_last;
  {
    const int pf = uni(s_pref[r_first]), wf = uni(s_pref[r_first + 1]) - pf;
    j_first = (int)((lo - (int64_t)U * pf + wf - 1) / wf);   // may be U: no unit of it in range
    const int pl = uni(s_pref[r_last]), wl = uni(s_pref[r_last + 1]) - pl;
    const int64_t je = (hi - (int64_t)U * pl + wl - 1) / wl;
    j_last = je < U ? (int)je : U;
  }

  const int gl = lane & 7, gw = lane >> 3;
  int rr = r_first;   // the next slot to consider
  for (;;) {
    // the staged set: the next slots of [rr, r_last] with units in the range, found with
    // one ballot over 64 slots (every wave finds the same), as many as the pool takes
    uint64_t m = 0;
    for (;;) {
      const int slot = rr + lane;
      bool has = false;
      if (slot <= r_last && s_pref[slot + 1] > s_pref[slot]) {
        const int a = slot == r_first ? j_first : 0, b = slot == r_last ? j_last : U;
        has = a < b;
      }
      m = __ballot(has);
      if (m != 0 || rr + kWave > r_last) break;
      rr += kWave;
    }
    if (m == 0) break;   // workgroup-uniform: the range is done
    if (threadIdx.x == 0) {
      int np = 0, cu = 0, off = 0;
      while (m != 0 && np < KP) {
        const int slot = rr + __builtin_ctzll(m);
        int cap = s_kap[slot] + s_lmb[slot] + 1;
        cap = cap < 1 ? 1 : (cap > LMAX ? LMAX : cap);   // the merge rejects counts beyond LMAX
        if (off + cap > kSpreadPool) break;
        m &= m - 1;
        const int a = slot == r_first ? j_first : 0, b = slot == r_last ? j_last : U;
        s_sl[np] = slot;
        s_ja[np] = a;
        s_cu[np] = cu;
        s_off[np] = off * nf;
        s_cap[np] = cap;
        cu += b - a;
        off += cap;
        ++np;
      }
      s_cu[np] = cu;
      s_np = np;
    }
    __syncthreads();
    const int np = uni(s_np);
    rr = uni(s_sl[np - 1]) + 1;
    // wave w < np merges staged particle w
    if (wave < np) {
      const int rw = uni(s_sl[wave]);
      const int64_t i = perm ? (int64_t)perm[rw] : rw;
      LayerStack *st = &s_stack[wave];
      const int L = merge_counts(p, i, true, uni(s_kap[rw]), uni(s_lmb[rw]), kc, km, LMAX, st, s.flags);
      if (L > 0) {
        const ColeCole cc = cole_cole(p, i);
        if (lane == 0) s_cc[wave] = cc;
        stage_h2<T>(st, L, s_h2[wave], lane);
      }
      if (lane == 0) {
        s_L[wave] = L;
        if (s_ja[wave] == 0) rim_layers[rw] = L;
      }
    }
    __syncthreads();
    // wavenumber tables of the frequency chunks the staged units need, one (particle,
    // frequency) pair per thread; particle sp's table of frequency f at s_off[sp] +
    // f s_cap[sp] (L <= capacity)
    for (int t = threadIdx.x; t < np * nf; t += blockDim.x) {
      const int sp = t / nf, f = t - sp * nf;
      const int L = s_L[sp];
      const int a = s_ja[sp], b = a + s_cu[sp + 1] - s_cu[sp];
      const int qa = a / nhg, qb = (b - 1) / nhg;
      if (L > 0 && f >= 8 * qa && f < 8 * qb + 8) {
        const LayerStack *st = &s_stack[sp];
        const K2Freq<T> kf = k2_freq<T>(s_omega[f], s_logw[f], s_cc[sp]);
        const int o = s_off[sp] + f * s_cap[sp];
        cplx<T> *k2 = s_k2 + o, *dk2 = s_dk2 + o;
        cplx<T> kl = k2_layer<T>(st, 0, kf);
        for (int l = 0; l < L; ++l) {
          k2[l] = kl;
          if (l + 1 < L) {
            const cplx<T> kn = k2_layer<T>(st, l + 1, kf);
            dk2[l] = kl - kn;
            kl = kn;
          }
        }
      }
    }
    __syncthreads();
    // the staged units, claimed one at a time by whichever wave is free
    const int nu = uni(s_cu[np]);
    const ExpConsts ek = exp_consts();
    for (;;) {
      int u = 0;
      if (lane == 0) u = atomicAdd(&s_next, 1);
      u = __builtin_amdgcn_readfirstlane(u);
      if (u >= nu) break;
      int sp = 0;
      while (sp + 1 < np && u >= uni(s_cu[sp + 1])) ++sp;
      const int L = uni(s_L[sp]);
      if (L == 0) continue;   // invalid particle: no terms
      const int jj = uni(s_ja[sp]) + u - uni(s_cu[sp]);
      const int q = jj / nhg, sidx = jj - q * nhg;
      const int jf = gw + 8 * q;
      const int o = uni(s_off[sp]) + jf * uni(s_cap[sp]);
      double v = 0.0;
      if (jf < nf)
        v = static_cast<double>(reflection_im<T>(to<T>(s_lam[gl + 8 * sidx]), s_k2 + o, s_dk2 + o, s_h2[sp], L,
                                                 s_phase, s_exp2, ek));
      // read once, by the second launch: streamed past L2 (its write-back at the end of the
      // kernel is shorter; 27.8 -> 27.0 us per launch on 256 particles, the second launch
      // 0.2 us longer)
      __builtin_nontemporal_store(v, &rim[(((int64_t)uni(s_sl[sp]) * nq + q) * nhg + sidx) * kWave + lane]);
    }
    __syncthreads();   // every claimed unit is done before the set is restaged
    if (threadIdx.x == 0) s_next = 0;
  }
}

// The evaluation is compiled for FP64 only: in FP32 the compiler contracts a few products
// of the recursion into FMAs differently here than in forward_kernel, so the terms would
// differ from the other shapes' in their last bits.

// One workgroup of n_q waves per slot: wave q adds chunk q's terms over the abscissae in
// the order of forward_kernel, then the first wave applies the gates and the likelihood.
__global__ __launch_bounds__(kWave * kMaxFreq / 8) void spread_finish_kernel(
    DevSystem s, DevParticles p, const int32_t *perm, const double *rim, const int32_t *rim_layers, double *resp,
    const double *y_obs, double *ll) {
  __shared__ double s_ck[kMaxHankel];
  __shared__ double s_eps2[kMaxGate];
  __shared__ double s_imh[kMaxFreq];
  extern __shared__ double s_K[];   // [n_gate][n_freq], dynamic
  const int nf = s.n_freq, ng = s.n_gate, nhp = s.n_hankel_pad;
  const int r = blockIdx.x;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int gl = lane & 7, gw = lane >> 3;
  const int nq = (nf + 7) >> 3, nhg = nhp >> 3;
  const int jf = gw + 8 * wave;
  // every global load of the workgroup is issued before the first wait: the first batch
  // of this wave's terms (read whatever the slot holds; used only for a valid particle),
  // the slot's layer count and particle, and the tables
  constexpr int kBatch = 16;   // terms in flight before the dependent sums
  const double *src = rim + ((int64_t)r * nq + wave) * nhg * kWave + lane;
  double v[kBatch];
#pragma unroll
  for (int t = 0; t < kBatch; ++t) v[t] = t < nhg ? src[(int64_t)t * kWave] : 0.0;
  const int L = rim_layers[r];
  const int64_t i = perm ? (int64_t)perm[r] : r;
  for (int t = threadIdx.x; t < nhp; t += blockDim.x) s_ck[t] = s.ck[t];
  for (int t = threadIdx.x; t < nf * ng; t += blockDim.x) s_K[t] = s.K[t];
  for (int t = threadIdx.x; t < ng; t += blockDim.x) s_eps2[t] = s.eps_an2[t];
  if (p.mask && p.mask[i] != p.mask_value) return;   // workgroup-uniform
  __syncthreads();
  if (L > 0) {
    double acc = 0.0;
    for (int s0 = 0; s0 < nhg; s0 += kBatch) {
      if (s0 > 0) {
#pragma unroll
        for (int t = 0; t < kBatch; ++t) v[t] = s0 + t < nhg ? src[(int64_t)(s0 + t) * kWave] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < kBatch; ++t)
        if (s0 + t < nhg) acc = __builtin_fma(s_ck[gl + 8 * (s0 + t)], v[t], acc);
    }
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    acc += __shfl_xor(acc, 4);
    if (gl == 0 && jf < nf) s_imh[jf] = acc;
  }
  __syncthreads();
  if (wave != 0) return;
  if (L > 0)
    gates_loglik(s, p, i, s_K, s_imh, s_eps2, resp, y_obs, ll, lane);
  else
    invalid_outputs(s, i, resp, ll, lane);
}

template <typename T>
static hipError_t launch_spread(const DevSystem &s, const DevParticles &p, int kc, int km, double *resp,
                                const double *y_obs, double *ll, const ForwardTiles &t, hipStream_t stream) {
  const int nq = (s.n_freq + 7) / 8;
  hipLaunchKernelGGL(spread_terms_kernel<T>, dim3((unsigned)t.n_cu), dim3(kWave * kSpreadWaves),
                     spread_table_bytes<T>(s), stream, s, p, kc, km, t.perm, t.rim, t.rim_layers);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(spread_finish_kernel, dim3((unsigned)p.n), dim3(kWave * nq),
                     sizeof(double) * s.n_freq * s.n_gate, stream, s, p, t.perm, t.rim, t.rim_layers, resp, y_obs,
                     ll);
  return hipGetLastError();
}

// Whether a launch over n particles can take the spread evaluation with these tiles.
static bool spread_ok(const ForwardTiles &t, int64_t n) {
  return t.rim && t.rim_layers && t.n_cu > 0 && n <= t.rim_n && n <= kSpreadMaxN;
}

int64_t spread_rim_doubles(const DevSystem &s, int64_t n) {
  return n * ((s.n_freq + 7) / 8) * (s.n_hankel_pad / 8) * kWave;
}

int64_t spread_max_particles() { return kSpreadMaxN; }

template <typename T>
static hipError_t spread_lds(const DevSystem &s, size_t *bytes) {
  hipFuncAttributes a1, a2;
  hipError_t e = hipFuncGetAttributes(&a1, reinterpret_cast<const void *>(&spread_terms_kernel<T>));
  if (e == hipSuccess) e = hipFuncGetAttributes(&a2, reinterpret_cast<const void *>(&spread_finish_kernel));
  if (e != hipSuccess) return e;
  const size_t b1 = a1.sharedSizeBytes + spread_table_bytes<T>(s);
  const size_t b2 = a2.sharedSizeBytes + sizeof(double) * s.n_freq * s.n_gate;
  *bytes = b1 > b2 ? b1 : b2;
  return hipSuccess;
}

// Dynamic LDS of one workgroup: K [n_gate][n_freq], plus the reflection terms
// [WPB][n_freq][n_hankel_pad] when the abscissa groups are split among the waves.
static size_t dynamic_lds(const DevSystem &s, int WPB, int P) {
  const int nq = (s.n_freq + 7) / 8;
  const int A = (P > 1 && P > nq) ? P / nq : 1;
  return sizeof(double) * (s.n_freq * s.n_gate + (A > 1 ? (size_t)WPB * s.n_freq * s.n_hankel_pad : 0));
}

template <typename T, int WPB, int P>
static hipError_t launch_t(const DevSystem &s, const DevParticles &p, int kc, int km, double *resp,
                           const double *y_obs, double *ll, const int32_t *perm, hipStream_t stream) {
  const int64_t blocks = (p.n + WPB - 1) / WPB;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((forward_kernel<T, WPB, P>), dim3((unsigned)blocks), dim3(kWave * WPB * P), dynamic_lds(s, WPB, P),
                     stream, s, p, kc, km, resp, y_obs, ll, perm);
  return hipGetLastError();
}

template <typename T, int WPB, int P>
static hipError_t lds_t(const DevSystem &s, size_t *bytes) {
  hipFuncAttributes attr;
  const hipError_t e = hipFuncGetAttributes(&attr, reinterpret_cast<const void *>(&forward_kernel<T, WPB, P>));
  if (e != hipSuccess) return e;
  *bytes = attr.sharedSizeBytes + dynamic_lds(s, WPB, P);
  return hipSuccess;
}

// Dispatch on the tile shape: F<T, WPB, P>(args...) for the compiled shapes.
#define RJSMC_TILE_DISPATCH(F, T, w, q, ...)                                  \
  do {                                                                        \
    if ((q) == 2 && (w) == 2) return F<T, 2, 2>(__VA_ARGS__);                 \
    if ((q) == 4 && (w) == 1) return F<T, 1, 4>(__VA_ARGS__);                 \
    if ((q) == 8 && (w) == 1) return F<T, 1, 8>(__VA_ARGS__);                 \
    if ((q) == 16 && (w) == 1) return F<T, 1, 16>(__VA_ARGS__);               \
    if ((q) != 1) return hipErrorInvalidValue;                                \
    if ((w) == 2) return F<T, 2, 1>(__VA_ARGS__);                             \
    if ((w) == 8) return F<T, 8, 1>(__VA_ARGS__);                             \
    if ((w) == 4) return F<T, 4, 1>(__VA_ARGS__);                             \
    return hipErrorInvalidValue;                                              \
  } while (0)

template <typename T>
static hipError_t launch_prec(const ForwardTiles &t, const DevSystem &s, const DevParticles &p, int kc, int km,
                              double *resp, const double *y_obs, double *ll, hipStream_t stream) {
  if (t.waves_per_particle == 0 && t.waves_per_block == kSpreadWaves) {
    if (p.n == 0) return hipSuccess;
    if (sizeof(T) == sizeof(double) && spread_ok(t, p.n))
      return launch_spread<double>(s, p, kc, km, resp, y_obs, ll, t, stream);
    return launch_t<T, 4, 1>(s, p, kc, km, resp, y_obs, ll, t.perm, stream);   // beyond the workspace
  }
  RJSMC_TILE_DISPATCH(launch_t, T, t.waves_per_block, t.waves_per_particle, s, p, kc, km, resp, y_obs, ll, t.perm,
                      stream);
}

template <typename T>
static hipError_t lds_prec(const DevSystem &s, int w, int q, size_t *bytes) {
  if (q == 0 && w == kSpreadWaves)   // FP64 only: not compiled for FP32
    return sizeof(T) == sizeof(double) ? spread_lds<double>(s, bytes) : hipErrorInvalidValue;
  RJSMC_TILE_DISPATCH(lds_t, T, w, q, s, bytes);
}

hipError_t launch_forward(const DevSystem &s, const DevParticles &p, int kc, int km, int precision,
                          double *resp, const double *y_obs, double *ll, hipStream_t stream,
                          const ForwardTiles &tiles) {
  if (precision == RJSMC_F32) return launch_prec<float>(tiles, s, p, kc, km, resp, y_obs, ll, stream);
  return launch_prec<double>(tiles, s, p, kc, km, resp, y_obs, ll, stream);
}

hipError_t forward_lds_bytes(const DevSystem &s, int precision, int waves_per_block, int waves_per_particle,
                             size_t *bytes) {
  if (precision == RJSMC_F32) return lds_prec<float>(s, waves_per_block, waves_per_particle, bytes);
  return lds_prec<double>(s, waves_per_block, waves_per_particle, bytes);
}

// ---- ordering of particles by layer capacity (counting sort, descending capacity)
// cnt[0..kCapBins) counts, cnt[kCapBins..2 kCapBins) cursors.  Bin b holds capacity
// kMaxLayers - b, so bin 0 (the deepest particles) is evaluated first.
namespace {
constexpr int kCapBins = kMaxLayers;

__device__ __forceinline__ int cap_bin(const DevParticles &p, int64_t i) {
  const int lam = p.layout == RJSMC_LAYOUT_DECOUPLED ? p.lambda[i] : 0;
  int cap = p.kappa[i] + lam + 1;
  cap = cap < 1 ? 1 : (cap > kMaxLayers ? kMaxLayers : cap);   // invalid counts: anywhere
  return kMaxLayers - cap;
}

__global__ void sort_zero_kernel(int *cnt) {
  if (threadIdx.x < 2 * kCapBins) cnt[threadIdx.x] = 0;
}

// Per wave: one ballot and one atomic per bin present.
__global__ __launch_bounds__(256) void sort_count_kernel(DevParticles p, int *cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const int bin = i < p.n ? cap_bin(p, i) : -1;
  uint64_t todo = __ballot(bin >= 0);
  while (todo) {
    const int leader = __builtin_ctzll(todo);
    const int b = __shfl(bin, leader);
    const uint64_t same = __ballot(bin == b);
    if (lane == leader) atomicAdd(&cnt[b], __popcll(same));
    todo &= ~same;
  }
}

__global__ void sort_scan_kernel(int *cnt) {
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int b = 0; b < kCapBins; ++b) {
      cnt[kCapBins + b] = acc;
      acc += cnt[b];
    }
  }
}

__global__ __launch_bounds__(256) void sort_scatter_kernel(DevParticles p, int *cnt, int32_t *perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const int bin = i < p.n ? cap_bin(p, i) : -1;
  uint64_t todo = __ballot(bin >= 0);
  while (todo) {
    const int leader = __builtin_ctzll(todo);
    const int b = __shfl(bin, leader);
    const uint64_t same = __ballot(bin == b);
    int base = 0;
    if (lane == leader) base = atomicAdd(&cnt[kCapBins + b], __popcll(same));
    base = __shfl(base, leader);
    if (bin == b) perm[base + __popcll(same & ((1ull << lane) - 1))] = (int32_t)i;
    todo &= ~same;
  }
}

// The whole sort in one workgroup, for small populations (where the four launches above
// are latency, not work): every thread loads the bins of its particles first (at most
// kSortRounds, in registers), counts them with LDS atomics, and after the scan places
// each particle at the slot an LDS atomic on its bin's cursor returns; the same counts and
// bin ends in cnt.
constexpr int kSortThreads = 1024;
constexpr int kSortRounds = 32;
constexpr int64_t kSortOneBlockMax = (int64_t)kSortThreads * kSortRounds;
__global__ __launch_bounds__(kSortThreads) void sort_block_kernel(DevParticles p, int *cnt, int32_t *perm) {
  __shared__ int hist[kCapBins], cur[kCapBins];
  if (threadIdx.x < kCapBins) hist[threadIdx.x] = 0;
  const int64_t n = p.n;
  int bins[kSortRounds];
#pragma unroll
  for (int k = 0; k < kSortRounds; ++k) {
    const int64_t i = (int64_t)k * kSortThreads + threadIdx.x;
    bins[k] = i < n ? cap_bin(p, i) : -1;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSortRounds; ++k)
    if (bins[k] >= 0) atomicAdd(&hist[bins[k]], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int b = 0; b < kCapBins; ++b) {
      cur[b] = acc;
      acc += hist[b];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSortRounds; ++k)
    if (bins[k] >= 0) perm[atomicAdd(&cur[bins[k]], 1)] = (int32_t)((int64_t)k * kSortThreads + threadIdx.x);
  __syncthreads();
  if (threadIdx.x < kCapBins) {
    cnt[threadIdx.x] = hist[threadIdx.x];
    cnt[kCapBins + threadIdx.x] = cur[threadIdx.x];   // the end of each bin
  }
}
}  // namespace

hipError_t launch_layer_sort(const DevParticles &p, int *cnt, int32_t *perm, hipStream_t stream) {
  if (p.n <= kSortOneBlockMax) {
    hipLaunchKernelGGL(sort_block_kernel, dim3(1), dim3(kSortThreads), 0, stream, p, cnt, perm);
    return hipGetLastError();
  }
  const int64_t blocks = (p.n + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sort_zero_kernel, dim3(1), dim3(64), 0, stream, cnt);
  hipLaunchKernelGGL(sort_count_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, cnt);
  hipLaunchKernelGGL(sort_scan_kernel, dim3(1), dim3(64), 0, stream, cnt);
  hipLaunchKernelGGL(sort_scatter_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, cnt, perm);
  return hipGetLastError();
}

}  // namespace rjsmc
