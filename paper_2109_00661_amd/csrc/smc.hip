// SMC primitives of adaptive RJSMC (Algorithm 1) for gfx950: prior initialisation,
// re-weighting with the tempering bisection and evidence update, within-model
// systematic resampling with the resampled copy, per-model proposal adaptation (also
// from recycled particles, Section 3.2.4), and the propose / accept halves of the
// RJ-MCMC mutation, including the adaptive birth of Appendix E.2 (the likelihood of
// each proposal is evaluated by the forward kernel in between).
//
// Weights, temperatures and evidence are FP64.  Resampling thresholds are exact
// integer arithmetic on weights quantised to 2^-60, so ancestor choices do not depend
// on summation order.  One workgroup owns one sounding for the reweight/resample step
// (its particles, log-likelihoods, model ids and cumulative weights live in LDS).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "cplx.h"
#include "rjsmc_internal.h"

namespace rjsmc {

// The step t of a re-weight or mutate call: from device memory when the caller keeps it
// there (replayed graphs), else the value passed.
template <typename A>
__device__ __forceinline__ int32_t step_of(const A &a) {
  return a.step_dev ? *a.step_dev : a.step;
}

__global__ void counter_add_kernel(int32_t *counter, int32_t delta) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter += delta;
}

hipError_t launch_counter_add(int32_t *counter, int32_t delta, hipStream_t stream) {
  hipLaunchKernelGGL(counter_add_kernel, dim3(1), dim3(64), 0, stream, counter, delta);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Philox4x32-10 ----
// Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11): ten rounds of two
// 32x32->64 multiplies with the Philox multipliers, with the key bumped by the Weyl
// constants between rounds.
constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;
constexpr uint32_t kDomainInit = 0x40000000u, kDomainResample = 0x80000000u;

__device__ __forceinline__ void philox10(uint32_t c[4], uint64_t seed) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c[0];
    const uint64_t p1 = (uint64_t)kPhiloxM1 * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = (uint32_t)p1;
    c[2] = n2;
    c[3] = (uint32_t)p0;
  }
}

__device__ __forceinline__ void bits53(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint64_t &x0, uint64_t &x1) {
  uint32_t c[4] = {c0, c1, c2, c3};
  philox10(c, seed);
  x0 = ((uint64_t)c[0] << 21) | (c[1] >> 11);
  x1 = ((uint64_t)c[2] << 21) | (c[3] >> 11);
}

// Two uniforms on (0, 1): (x + 0.5) 2^-53.
__device__ __forceinline__ void uniforms(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         double &u0, double &u1) {
  uint64_t x0, x1;
  bits53(seed, c0, c1, c2, c3, x0, x1);
  u0 = ((double)x0 + 0.5) * 0x1.0p-53;
  u1 = ((double)x1 + 0.5) * 0x1.0p-53;
}

// Box-Muller: first normal of the pair.
__device__ __forceinline__ double normal0(double u1, double u2) {
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586477 * u2);
}

// lo + (hi - lo) u with each operation rounded separately (no fused multiply-add).
__device__ __forceinline__ double affine(double lo, double hi, double u) {
#pragma clang fp contract(off)
  return lo + (hi - lo) * u;
}

// a + b c with the product rounded before the sum.
__device__ __forceinline__ double madd_rn(double a, double b, double c) {
#pragma clang fp contract(off)
  return a + b * c;
}

// ------------------------------------------------------------------------ prior ------
__global__ __launch_bounds__(256) void init_prior_kernel(DevParticlesW p, SmcShape sh, rjsmc_prior pr,
                                                         uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const int64_t S = p.stride;
  const int kc = sh.kc, km = sh.km;
  auto u_at = [&](int idx) {
    double a, b;
    uniforms(seed, (uint32_t)i, 0u, (uint32_t)(idx >> 1), kDomainInit, a, b);
    return (idx & 1) ? b : a;
  };
  int kap = (int)(u_at(0) * (double)(kc + 1));
  kap = kap > kc ? kc : kap;
  int lam = (int)(u_at(1) * (double)(km + 1));
  lam = lam > km ? km : lam;
  p.kappa[i] = kap;
  p.lambda[i] = lam;
  p.phi_b[i] = affine(pr.phi_lo, pr.phi_hi, u_at(2));
  p.log10_tau[i] = affine(pr.ltau_lo, pr.ltau_hi, u_at(3));
  p.c[i] = affine(pr.c_lo, pr.c_hi, u_at(4));
  double z[kMaxLayers];
  // conductivity interfaces: sorted depths, properties in draw order
  for (int j = 0; j < kap; ++j) {
    const double v = sh.z_max * u_at(6 + j);
    int t = j;
    while (t > 0 && z[t - 1] > v) {
      z[t] = z[t - 1];
      --t;
    }
    z[t] = v;
  }
  for (int j = 0; j < kc; ++j) {
    p.z_cond[(int64_t)j * S + i] = j < kap ? z[j] : 0.0;
    p.phi[(int64_t)j * S + i] = j < kap ? affine(pr.phi_lo, pr.phi_hi, u_at(6 + kc + j)) : 0.0;
  }
  const int base2 = 6 + 2 * kc;
  for (int j = 0; j < lam; ++j) {
    const double v = sh.z_max * u_at(base2 + j);
    int t = j;
    while (t > 0 && z[t - 1] > v) {
      z[t] = z[t - 1];
      --t;
    }
    z[t] = v;
  }
  for (int j = 0; j < km; ++j) {
    p.z_charg[(int64_t)j * S + i] = j < lam ? z[j] : 0.0;
    p.m[(int64_t)j * S + i] = j < lam ? affine(pr.m_lo, pr.m_hi, u_at(base2 + km + j)) : 0.0;
  }
}

hipError_t launch_init_prior(const DevParticlesW &p, const SmcShape &sh, const rjsmc_prior &pr, uint64_t seed,
                             hipStream_t stream) {
  const int64_t blocks = (p.n + 255) / 256;
  hipLaunchKernelGGL(init_prior_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, sh, pr, seed);
  return hipGetLastError();
}

// ----------------------------------------------------------- reweight / resample -----
constexpr int kRwThreads = 512;
constexpr int kRwWaves = kRwThreads / kWave;
constexpr int kMaxPerSounding = 2048;         // register-resident runs (two kernels)
constexpr int kMaxPerSoundingLarge = RJSMC_MAX_PER_SOUNDING;   // LDS-resident runs
constexpr int kMaxModels = 128;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// The temperature increment is the lower end of the bracket that 60 halvings of
// (0, 1 - gamma] leave, each halving keeping the half whose lower end passes the test
// TESS >= alpha N.  TESS does not increase with the increment (tilting the weights further
// towards the larger log-likelihoods can only concentrate them), so a midpoint at or below
// a point that passed also passes, and one at or above a point that failed also fails.
// The search therefore first narrows a bracket (a, b) around the root with Newton steps
// on ln TESS in ln(increment), falling back to a geometric halving whenever a step leaves
// the bracket, then replays the 60 halvings, evaluating TESS only at the midpoints that
// fall inside the bracket and taking the others from its ends.  Typically a dozen
// evaluations replace sixty; the replay makes the same decisions as a plain bisection
// wherever TESS differs from the target by more than its rounding.
//
// Each live model's members (sorted order) are cut into runs of R consecutive members
// (the model's last run may be shorter), one run per lane, runs in model order across the
// workgroup; R is the least length whose runs fit the 512 lanes (at most 5 for 2,048
// members and 128 models).  A lane keeps its run's x values in registers for the whole
// search; an evaluation is then: the lane's exponentials and their sums, a segmented scan
// over the lanes of each wave (a model's lanes are contiguous), the carries of models that
// span waves, and the sum over models of the per-model ESS.  All sums are taken in a
// fixed order, so every thread obtains the same TESS and takes the same decisions.
constexpr int kEvalK = 2;        // increments per evaluation at most
constexpr int kRunMax = 5;
constexpr int kNewtonMax = 16;
static_assert(kMaxPerSounding + kMaxModels * (kRunMax - 1) <= kRwThreads * kRunMax, "runs of 5 always fit");

struct RwShared {
  union {
    double ll[kMaxPerSounding];                       // particle order, until x is formed
    uint64_t cum[kMaxPerSounding];                    // cumulative weights, after the search
  } u;
  double x[kMaxPerSounding];        // sorted order: ll - max of the model (-inf: dead model)
  union {
    int wc[kRwWaves][kMaxModels];   // per-wave model counts, then running placement offsets
    int16_t anc_l[kMaxPerSounding]; // ancestor of each particle (index within the sounding)
  } v;
  int16_t idx[kMaxPerSounding];     // particles sorted by (model, index)
  uint8_t mod[kMaxPerSounding];
  int cnt[kMaxModels], base[kMaxModels], rb[kMaxModels + 1];
  double mx[kMaxModels], s1[kMaxModels];
  uint64_t U[kMaxModels];
  double tail[kRwWaves][2 * kEvalK];   // wave-end partial sums of the scanned values
  double wess[kRwWaves][kEvalK];        // per-wave sums of the models' ESS (or ESS, derivative)
  double e2[kExp2N];                // 2^(j/256), the table of exp_tab
  int run_len;
};

// Large soundings (up to kMaxPerSoundingLarge = 10,240 members, 13 bytes of LDS each):
// the log-likelihoods are written straight into sorted order (x holds ll, then ll minus
// the model's maximum), the cumulative weights overwrite x in place, and the runs are
// read from LDS at every evaluation instead of being held in registers.
struct RwSharedLarge {
  union {
    double x[kMaxPerSoundingLarge];       // sorted order: ll, then ll - max of the model
    uint64_t cum[kMaxPerSoundingLarge];   // cumulative weights, after the search
  } u;
  union {
    int wc[kRwWaves][kMaxModels];
    int16_t anc_l[kMaxPerSoundingLarge];
  } v;
  int16_t idx[kMaxPerSoundingLarge];
  uint8_t mod[kMaxPerSoundingLarge];
  int cnt[kMaxModels], base[kMaxModels], rb[kMaxModels + 1];
  double mx[kMaxModels], s1[kMaxModels];
  uint64_t U[kMaxModels];
  double tail[kRwWaves][2 * kEvalK];
  double wess[kRwWaves][kEvalK];
  double e2[kExp2N];
  int run_len;
};
// sorted-order values of either layout
__device__ __forceinline__ double *xs_of(RwShared &sm) { return sm.x; }
__device__ __forceinline__ double *xs_of(RwSharedLarge &sm) { return sm.u.x; }
__device__ __forceinline__ const double *xs_of(const RwShared &sm) { return sm.x; }
__device__ __forceinline__ const double *xs_of(const RwSharedLarge &sm) { return sm.u.x; }

// A lane's run: model m (-1: no run), nv members with values x, seg the steps of the
// segmented wave scan (dpp_scan_step) whose source lane holds a run of the same model,
// fin on the model's last lane, w0 the wave of the model's first lane.
struct RunLane {
  int m, nv, seg, w0;
  bool fin;
  int xoff;                 // offset of the run's first value in sorted order
  double x[kRunMax];        // the run's values (register-resident runs only)
};

template <bool LOAD, typename SM>
__device__ __forceinline__ RunLane run_of_lane(const SM &sm, int M) {
  RunLane r;
  r.xoff = 0;
  const int t = threadIdx.x, lane = t & (kWave - 1);
  r.m = -1;
  r.nv = 0;
  r.seg = 0;
  r.w0 = 0;
  r.fin = false;
#pragma unroll
  for (int j = 0; j < kRunMax; ++j) r.x[j] = 0.0;
  if (t >= sm.rb[M]) return r;
  int lo = 0, hi = M;                 // rb[lo] <= t < rb[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (sm.rb[mid] <= t)
      lo = mid;
    else
      hi = mid;
  }
  const int R = sm.run_len;
  const int m = lo, m0 = sm.rb[m], m1 = sm.rb[m + 1];
  const int q0 = (t - m0) * R, rem = sm.cnt[m] - q0;
  r.m = m;
  r.nv = rem < R ? rem : R;
  r.fin = t == m1 - 1;
  r.w0 = m0 / kWave;
  const int row = lane >> 4, rl = lane & 15, wb = t - lane;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (rl >= (1 << k) && t - (1 << k) >= m0) r.seg |= 1 << k;
  if ((row == 1 || row == 3) && wb + 16 * row - 1 >= m0) r.seg |= 1 << 4;
  if (row >= 2 && wb + 31 >= m0) r.seg |= 1 << 5;
  r.xoff = sm.base[m] + q0;
  if (LOAD) {
    const double *xs = xs_of(sm) + r.xoff;
#pragma unroll
    for (int j = 0; j < kRunMax; ++j)
      if (j < r.nv) r.x[j] = xs[j];
  }
  return r;
}

// v of another lane by a DPP move (0 where the pattern has no source): CTRL 0x111 + j is
// lane - 2^j of the same 16-lane row, 0x142 the last lane of the previous row, 0x143
// lane 31.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum of v over the lanes of a wave, left in lane 63: the unsegmented form of the scan
// below (sources outside the pattern read 0).
template <int V>
__device__ __forceinline__ void wave_total(double (&v)[V]) {
  auto step = [&](auto ctrl) {
    constexpr int C = decltype(ctrl)::value;
#pragma unroll
    for (int q = 0; q < V; ++q) v[q] += dpp_f64<C>(v[q]);
  };
  step(std::integral_constant<int, 0x111>{});
  step(std::integral_constant<int, 0x112>{});
  step(std::integral_constant<int, 0x114>{});
  step(std::integral_constant<int, 0x118>{});
  step(std::integral_constant<int, 0x142>{});
  step(std::integral_constant<int, 0x143>{});
}

// Inclusive scan of v over the lanes of a wave, restarted where the model changes:
// row-local steps from lanes -1, -2, -4, -8, then the previous row's last lane (rows 1
// and 3) and lane 31 (rows 2 and 3); seg bit j says whether step j's source lane holds
// the same model.  A fixed order of additions, so the sums are reproducible.
template <int V>
__device__ __forceinline__ void seg_scan(double (&v)[V], int seg) {
  auto step = [&](auto ctrl, int bit) {
    constexpr int C = decltype(ctrl)::value;
    const bool take = (seg >> bit) & 1;
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const double t = dpp_f64<C>(v[q]);
      if (take) v[q] += t;
    }
  };
  step(std::integral_constant<int, 0x111>{}, 0);
  step(std::integral_constant<int, 0x112>{}, 1);
  step(std::integral_constant<int, 0x114>{}, 2);
  step(std::integral_constant<int, 0x118>{}, 3);
  step(std::integral_constant<int, 0x142>{}, 4);
  step(std::integral_constant<int, 0x143>{}, 5);
}

// TESS at K increments (all threads call, all return the same values).  With DER (K = 1)
// also its derivative in the increment, from the per-model sums A = sum w, B = sum w^2,
// A1 = sum x w, B1 = sum x w^2:  d(A^2/B)/d dg = 2 A (A1 B - A B1) / B^2.  With keep,
// sm.s1[m] = A of model m at dg[0].  RM bounds the run length.
template <int K, int RM, bool DER, typename SM>
__device__ __forceinline__ void eval_tess(SM &sm, const RunLane &r, const double (&dg)[K], double (&tess)[K],
                                          double &dtess, int M, bool keep) {
  static_assert(K <= kEvalK && (!DER || K == 1), "evaluation shape");
  constexpr int V = DER ? 4 : 2 * K;     // scanned values: A[K], B[K] (, A1, B1)
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  double v[V];
#pragma unroll
  for (int q = 0; q < V; ++q) v[q] = 0.0;
  auto add = [&](double xj) {
#pragma unroll
    for (int c = 0; c < K; ++c) {
      const double w = exp_tab(dg[c] * xj, sm.e2);
      v[c] += w;
      v[K + c] = fma(w, w, v[K + c]);
      if (DER) {
        const double xw = xj * w;
        v[2] += xw;
        v[3] = fma(xw, w, v[3]);
      }
    }
  };
  if (RM > 0) {
#pragma unroll
    for (int j = 0; j < (RM > 0 ? RM : 1); ++j)
      if (j < r.nv) add(r.x[j]);
  } else {                              // runs read from LDS (large soundings)
    const double *xs = xs_of(sm) + r.xoff;
    for (int j = 0; j < r.nv; ++j) add(xs[j]);
  }
  seg_scan<V>(v, r.seg);
  if (lane == kWave - 1)
#pragma unroll
    for (int q = 0; q < V; ++q) sm.tail[wave][q] = v[q];
  __syncthreads();
  constexpr int S = DER ? 2 : K;        // per-model terms: ESS at each increment (, derivative)
  double e[S];
#pragma unroll
  for (int c = 0; c < S; ++c) e[c] = 0.0;
  if (r.fin) {
    double t[V];                      // earlier waves' parts of the model, in wave order
#pragma unroll
    for (int q = 0; q < V; ++q) t[q] = 0.0;
    for (int w2 = r.w0; w2 < wave; ++w2)
#pragma unroll
      for (int q = 0; q < V; ++q) t[q] += sm.tail[w2][q];
#pragma unroll
    for (int q = 0; q < V; ++q) t[q] += v[q];
#pragma unroll
    for (int c = 0; c < K; ++c) e[c] = t[c] * t[c] / t[K + c];
    if (DER) e[S - 1] = 2.0 * t[0] * (t[2] * t[1] - t[0] * t[3]) / (t[1] * t[1]);
    if (keep) sm.s1[r.m] = t[0];
  }
  // the models' terms summed over each wave's lanes (models in lane order), then the
  // waves' sums in wave order
  wave_total<S>(e);
  if (lane == kWave - 1)
#pragma unroll
    for (int c = 0; c < S; ++c) sm.wess[wave][c] = e[c];
  __syncthreads();
  double acc[S];
#pragma unroll
  for (int c = 0; c < S; ++c) acc[c] = 0.0;
#pragma unroll
  for (int w2 = 0; w2 < kRwWaves; ++w2)
#pragma unroll
    for (int c = 0; c < S; ++c) acc[c] += sm.wess[w2][c];
#pragma unroll
  for (int c = 0; c < K; ++c) tess[c] = acc[c];
  dtess = DER ? acc[S - 1] : 0.0;
}

// ln(f / t) for the Newton steps: the series 2 atanh(s), s = (f - t) / (f + t), when
// f / t is near 1 (where the steps must be accurate; the terms beyond s^19 are below
// 1e-19 relative), a single-precision logarithm elsewhere (far from the root a step only
// needs its direction and rough size; every decision comes from an evaluation).
__device__ __forceinline__ double ln_ratio(double f, double t) {
  const double s = (f - t) / (f + t);
  if (fabs(s) < 0.125) {
    const double s2 = s * s;
    double p = 1.0 / 19.0;
    p = fma(p, s2, 1.0 / 17.0);
    p = fma(p, s2, 1.0 / 15.0);
    p = fma(p, s2, 1.0 / 13.0);
    p = fma(p, s2, 1.0 / 11.0);
    p = fma(p, s2, 1.0 / 9.0);
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    p = fma(p, s2, 1.0);
    return 2.0 * s * p;
  }
  return (double)__logf((float)(f / t));
}

// The increment (see the search description above); full when the whole remaining step
// 1 - gamma = H passes.  On return sm.s1 holds the per-model weight sums at the increment.
template <int RM, typename SM>
__device__ double next_increment(SM &sm, const RunLane &r, double H, double target, int M, bool &full) {
  double t1[1], dt;
  {
    const double d0[1] = {H};
    eval_tess<1, RM, true>(sm, r, d0, t1, dt, M, true);
  }
  full = t1[0] >= target;
  if (full) return H;
  double a = 0.0, b = H;                        // TESS(a) >= target (when a > 0), TESS(b) < target
  // current point: u ~ ln d, TESS f and its derivative df; ua, ub ~ ln a, ln b (the
  // logarithms only steer the steps: the bracket itself is a, b)
  const double lnH = (double)__logf((float)H);
  const double u_min = lnH - 62.0 * 0.69314718055994531;   // below every halving midpoint
  double u = lnH, d = H, f = t1[0], df = dt, ua = u_min, ub = u;
  bool converged = false;
  double step = 0.0;
  for (int it = 0; it < kNewtonMax && b - a > H * 0x1p-61; ++it) {
    double un = u - ln_ratio(f, target) * f / (d * df);
    if (fabs(un - u) < 1e-14) {                 // the root is within |un - u| of the current point
      converged = true;
      step = un - u;
      break;
    }
    if (!(un > ua && un < ub)) {                 // outside the bracket, or NaN: before any
      // point has passed, step 10 below the failing end (increments within e^10 of the
      // remaining step are the common case), else halve the bracket geometrically
      const double down = ub - 10.0;
      un = a == 0.0 && down > 0.5 * (ua + ub) ? down : 0.5 * (ua + ub);
    }
    const double dn = exp_tab(un, sm.e2);      // un < ub <= 0
    if (!(dn > a && dn < b)) break;             // no representable point left inside
    const double dd[1] = {dn};
    eval_tess<1, RM, true>(sm, r, dd, t1, dt, M, false);
    if (t1[0] >= target) {
      a = dn;
      ua = un;
    } else {
      b = dn;
      ub = un;
    }
    u = un;
    d = dn;
    f = t1[0];
    df = dt;
  }
  if (converged && b - a > H * 0x1p-61) {
    // tighten the bracket around the converged estimate
    const double dn = d * (1.0 + step), del = 2.0 * fabs(step) + 0x1p-49;
    double pd[2] = {dn * (1.0 - del), dn * (1.0 + del)}, tp[2], unused;
    pd[0] = pd[0] > a ? pd[0] : a;
    pd[1] = pd[1] < b ? pd[1] : b;
    eval_tess<2, RM, false>(sm, r, pd, tp, unused, M, false);
    if (tp[0] >= target && pd[0] > a) a = pd[0];
    if (tp[1] < target && pd[1] < b) b = pd[1];
  }
  // the 60 halvings, evaluating only inside the bracket
  double lo = 0.0, hi = H;
  for (int k = 0; k < 60; ++k) {
    const double c = 0.5 * (lo + hi);
    bool pass;
    if (a > 0.0 && c <= a) {
      pass = true;
    } else if (c >= b) {
      pass = false;
    } else {
      const double cc[1] = {c};
      double tc[1], unused;
      eval_tess<1, RM, false>(sm, r, cc, tc, unused, M, false);
      pass = tc[0] >= target;
    }
    if (pass)
      lo = c;
    else
      hi = c;
  }
  return lo;
}

// floor(((j << 53) + U) * T / (n << 53)) for j < n <= 2^14, U < 2^53, T < 2^61.  A =
// (j << 53) + U takes up to 67 bits (a_hi, a_lo); A T < n 2^53 T < 2^128.
__device__ __forceinline__ uint64_t sys_threshold(uint64_t j, uint64_t U, uint64_t T, uint64_t n) {
  const uint64_t a_lo = (j << 53) + U;                      // mod 2^64
  const uint64_t a_hi = (j >> 11) + (a_lo < U ? 1u : 0u);   // with the carry of the addition
  const uint64_t lo = a_lo * T, hi = __umul64hi(a_lo, T) + a_hi * T;
  // P1 = floor(A T / 2^53) as (p_hi, p_lo)
  const uint64_t p_lo = (hi << 11) | (lo >> 53);
  const uint64_t p_hi = hi >> 53;
  // long division of (p_hi, p_lo) by n in 32-bit digits
  uint64_t r = p_hi % n;
  uint64_t t1 = (r << 32) | (p_lo >> 32);
  const uint64_t q1 = t1 / n;
  r = t1 % n;
  const uint64_t t2 = (r << 32) | (p_lo & 0xffffffffull);
  const uint64_t q2 = t2 / n;
  return (q1 << 32) | q2;
}

// Lanes of the wave that hold the same model m (valid lanes only): nbits ballots.
__device__ __forceinline__ uint64_t same_model_lanes(int m, bool valid, int nbits) {
  uint64_t same = __ballot(valid);
  for (int b = 0; b < nbits; ++b) {
    const bool bit = (m >> b) & 1;
    const uint64_t ones = __ballot(valid && bit);
    same &= bit ? ones : ~ones;
  }
  return same;
}

__device__ __forceinline__ int wave_scan_incl(int v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

// Element at a 32-bit byte offset from a uniform base (lets the compiler use the
// scalar-base, vector-offset addressing of global memory instructions).
template <typename T>
__device__ __forceinline__ T ld_off(const T *base, uint32_t bytes) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + bytes);
}
template <typename T>
__device__ __forceinline__ void st_off(T *base, uint32_t bytes, T v) {
  *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + bytes) = v;
}

// out[i] = in[anc_l[i]] for the members i = first + tid + k * kRwThreads of the sounding,
// every row of the population, ll, and the global ancestor index.  Rows are addressed from the
// sounding's first element (a uniform base) with 32-bit byte offsets.  Loads are
// unconditional (a lane past the sounding reads member 0) and issued in groups before
// their stores, which are the only predicated accesses, so a group's loads are in flight
// together.
constexpr int kCopyPer = kMaxPerSounding / kRwThreads;
// CP members per thread (first + tid + k kRwThreads, k < CP), RB layer rows per batch of
// loads.
template <int CP, int RB, typename SM>
__device__ __forceinline__ void copy_resampled(const SM &sm, const DevParticles &in,
                                               const double *__restrict__ ll_in, const DevParticlesW &out,
                                               double *__restrict__ ll_out, int32_t *__restrict__ anc, int64_t off,
                                               int N, int rows_c, int rows_m, int rows_zm, int first = 0) {
  const int tid = threadIdx.x;
  const int64_t Si = in.stride, So = out.stride;
  uint32_t src[CP], dst[CP];   // member indices within the sounding
  bool ok[CP];
#pragma unroll
  for (int k = 0; k < CP; ++k) {
    const int i = first + tid + k * kRwThreads;
    ok[k] = i < N;
    dst[k] = ok[k] ? (uint32_t)i : 0u;
    src[k] = ok[k] ? (uint32_t)sm.v.anc_l[i] : 0u;
  }
  {
    int32_t ka[CP], la[CP];
    double lv[CP];
#pragma unroll
    for (int k = 0; k < CP; ++k) {
      ka[k] = ld_off(in.kappa + off, src[k] * 4u);
      la[k] = in.lambda ? ld_off(in.lambda + off, src[k] * 4u) : 0;
      lv[k] = ld_off(ll_in + off, src[k] * 8u);
    }
#pragma unroll
    for (int k = 0; k < CP; ++k)
      if (ok[k]) {
        st_off(anc + off, dst[k] * 4u, (int32_t)(off + src[k]));
        st_off(out.kappa + off, dst[k] * 4u, ka[k]);
        if (out.lambda) st_off(out.lambda + off, dst[k] * 4u, la[k]);
        st_off(ll_out + off, dst[k] * 8u, lv[k]);
      }
  }
  {
    double pb[CP], lt[CP], cc[CP];
#pragma unroll
    for (int k = 0; k < CP; ++k) {
      pb[k] = ld_off(in.phi_b + off, src[k] * 8u);
      lt[k] = ld_off(in.log10_tau + off, src[k] * 8u);
      cc[k] = ld_off(in.c + off, src[k] * 8u);
    }
#pragma unroll
    for (int k = 0; k < CP; ++k)
      if (ok[k]) {
        st_off(out.phi_b + off, dst[k] * 8u, pb[k]);
        st_off(out.log10_tau + off, dst[k] * 8u, lt[k]);
        st_off(out.c + off, dst[k] * 8u, cc[k]);
      }
  }
  // layer rows of one or two fields, RB rows of each per batch of loads (with four members
  // per thread more loads in flight would cost the registers of a third workgroup per CU;
  // with one, a sounding's copy is a chain of load round trips that batches shorten)
  auto rows_of = [&](const double *ia, const double *ib, double *oa, double *ob, int rows) {
    for (int r0 = 0; r0 < rows; r0 += RB) {
      double v[RB][2][CP];
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const int r = r0 + b;
#pragma unroll
        for (int k = 0; k < CP; ++k) {
          v[b][0][k] = r < rows ? ld_off(ia + r * Si + off, src[k] * 8u) : 0.0;
          v[b][1][k] = ib && r < rows ? ld_off(ib + r * Si + off, src[k] * 8u) : 0.0;
        }
      }
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const int r = r0 + b;
        if (r >= rows) continue;
#pragma unroll
        for (int k = 0; k < CP; ++k)
          if (ok[k]) {
            st_off(oa + r * So + off, dst[k] * 8u, v[b][0][k]);
            if (ob) st_off(ob + r * So + off, dst[k] * 8u, v[b][1][k]);
          }
      }
    }
  };
  rows_of(in.phi, in.z_cond, out.phi, out.z_cond, rows_c);
  if (rows_zm == rows_m)
    rows_of(in.m, in.z_charg, out.m, out.z_charg, rows_m);
  else
    rows_of(in.m, nullptr, out.m, nullptr, rows_m);
}

// One workgroup per sounding: re-weight, evidence, within-model resampling, and the
// resampled population written to out (each particle copied from its ancestor).  KIND 0:
// at most 512 particles per sounding, so every run is a single member (the evaluation
// code is then compiled for runs of one); KIND 1: at most 2,048, runs of up to five
// members in registers; KIND 2: at most 10,240, the large layout (runs read from LDS).
template <int KIND>
__global__ __launch_bounds__(kRwThreads) void reweight_resample_kernel(SmcShape sh, rjsmc_reweight_args a,
                                                                       DevParticles in, const double *ll_in,
                                                                       DevParticlesW out, double *ll_out,
                                                                       double *gamma, double *log_z,
                                                                       int32_t *active, int32_t *anc, int *flags,
                                                                       const double *exp2t) {
  constexpr bool LARGE = KIND == 2;
  // the copy: one member per thread and 8 rows per batch of loads for at most kRwThreads
  // members (KIND 0), else four members per thread, one row per batch
  constexpr int kCP = KIND == 0 ? 1 : kCopyPer, kRB = KIND == 0 ? 8 : 1;
  using SM = typename std::conditional<LARGE, RwSharedLarge, RwShared>::type;
  constexpr int NMAX = LARGE ? kMaxPerSoundingLarge : kMaxPerSounding;
  __shared__ SM sm;
  double *xs = xs_of(sm);
  const bool dec = in.layout == RJSMC_LAYOUT_DECOUPLED;
  const int rows_c = sh.kc, rows_m = dec ? sh.km : sh.kc + 1, rows_zm = dec ? sh.km : 0;
  const int s = blockIdx.x;
  const int N = (int)(in.n_per_sounding > 0 ? in.n_per_sounding : in.n);
  const int64_t off = (int64_t)s * N;
  const int M = sh.n_models;
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid & (kWave - 1);
  const double g0 = gamma[s];
  if (N > NMAX) return;                 // the host never launches this (rejected before)
  if (!(g0 < 1.0)) {
    for (int i = tid; i < N; i += kRwThreads) sm.v.anc_l[i] = (int16_t)i;
    __syncthreads();
    for (int first = 0; first < N; first += kCP * kRwThreads)
      copy_resampled<kCP, kRB>(sm, in, ll_in, out, ll_out, anc, off, N, rows_c, rows_m, rows_zm, first);
    if (tid == 0 && active) active[s] = 0;
    return;
  }
  // counts, models and log-likelihoods (loads first, then the LDS writes); the large
  // layout re-reads the log-likelihoods when it places the particles in sorted order
  for (int first = 0; first < N; first += kCopyPer * kRwThreads) {
    int kap[kCopyPer], lam[kCopyPer];
    double llv[kCopyPer];
#pragma unroll
    for (int k = 0; k < kCopyPer; ++k) {
      const int i = first + tid + k * kRwThreads;
      if (i < N) {
        kap[k] = in.kappa[off + i];
        lam[k] = in.lambda[off + i];
        if (!LARGE) llv[k] = ll_in[off + i];
      }
    }
#pragma unroll
    for (int k = 0; k < kCopyPer; ++k) {
      const int i = first + tid + k * kRwThreads;
      if (i < N) {
        const bool okc = kap[k] >= 0 && kap[k] <= sh.kc && lam[k] >= 0 && lam[k] <= sh.km;
        // a particle with counts outside the capacities is flagged and given -inf weight
        if constexpr (!LARGE) sm.u.ll[i] = okc ? llv[k] : -HUGE_VAL;
        if (!okc) atomicOr(flags, kFlagCapacity);
        sm.mod[i] = (uint8_t)(okc ? kap[k] * (sh.km + 1) + lam[k] : 0);
      }
    }
  }
  for (int t = tid; t < kRwWaves * kMaxModels; t += kRwThreads) (&sm.v.wc[0][0])[t] = 0;
  for (int t = tid; t < kExp2N; t += kRwThreads) sm.e2[t] = exp2t[t];
  __syncthreads();
  // stable counting sort by model: wave w takes a contiguous range of 64-particle chunks,
  // counts its members per model, then places them in order behind the earlier waves'
  const int nbits = M > 1 ? 32 - __clz(M - 1) : 0;
  const int n_chunks = (N + kWave - 1) / kWave, cpw = (n_chunks + kRwWaves - 1) / kRwWaves;
  const int ch0 = wave * cpw, ch1 = min(n_chunks, ch0 + cpw);
  const uint64_t below = (1ull << lane) - 1;
  for (int ch = ch0; ch < ch1; ++ch) {
    const int i = ch * kWave + lane;
    const bool v = i < N;
    const int m = v ? sm.mod[i] : 0;
    const uint64_t same = same_model_lanes(m, v, nbits);
    if (v && (same & below) == 0) sm.v.wc[wave][m] += __popcll(same);
  }
  __syncthreads();
  for (int m = tid; m < M; m += kRwThreads) {
    int acc = 0;
#pragma unroll
    for (int w = 0; w < kRwWaves; ++w) {
      const int c = sm.v.wc[w][m];
      sm.v.wc[w][m] = acc;
      acc += c;
    }
    sm.cnt[m] = acc;
    sm.mx[m] = -HUGE_VAL;
  }
  __syncthreads();
  if (wave == 0) {
    const int c0 = lane < M ? sm.cnt[lane] : 0, c1 = lane + kWave < M ? sm.cnt[lane + kWave] : 0;
    const int i0 = wave_scan_incl(c0);
    const int i1 = wave_scan_incl(c1) + __shfl(i0, kWave - 1);
    if (lane < M) sm.base[lane] = i0 - c0;
    if (lane + kWave < M) sm.base[lane + kWave] = i1 - c1;
  }
  __syncthreads();
  for (int ch = ch0; ch < ch1; ++ch) {
    const int i = ch * kWave + lane;
    const bool v = i < N;
    const int m = v ? sm.mod[i] : 0;
    const uint64_t same = same_model_lanes(m, v, nbits);
    double llp = 0.0;
    if (LARGE && v) {                  // the log-likelihood for its sorted position
      const int kk = in.kappa[off + i], lk = in.lambda[off + i];
      const bool okc = kk >= 0 && kk <= sh.kc && lk >= 0 && lk <= sh.km;
      llp = okc ? ll_in[off + i] : -HUGE_VAL;
    }
    if (v) {
      const int pos = sm.base[m] + sm.v.wc[wave][m] + __popcll(same & below);
      if (pos >= 0 && pos < N) {
        sm.idx[pos] = (int16_t)i;
        if (LARGE) xs[pos] = llp;
      }
      if ((same & below) == 0) sm.v.wc[wave][m] += __popcll(same);
    }
  }
  __syncthreads();
  // per-model maxima and resampling uniforms
  for (int m = wave; m < M; m += kRwWaves) {
    const int n = sm.cnt[m];
    double v = -HUGE_VAL;
    for (int q = lane; q < n; q += kWave) {
      if constexpr (LARGE)
        v = fmax(v, xs[sm.base[m] + q]);
      else
        v = fmax(v, sm.u.ll[sm.idx[sm.base[m] + q]]);
    }
    v = wave_max(v);
    if (lane == 0) {
      sm.mx[m] = v;
      uint64_t x0, x1;
      bits53(a.seed, (uint32_t)s, (uint32_t)step_of(a), (uint32_t)m, kDomainResample, x0, x1);
      sm.U[m] = x0;
    }
  }
  __syncthreads();
  // x in sorted order (the particle-order ll is not needed after this)
  for (int pos = tid; pos < N; pos += kRwThreads) {
    const int m = sm.mod[sm.idx[pos]];
    const double mx = sm.mx[m];
    double llv;
    if constexpr (LARGE)
      llv = xs[pos];
    else
      llv = sm.u.ll[sm.idx[pos]];
    xs[pos] = mx > -HUGE_VAL ? llv - mx : -HUGE_VAL;
  }
  // run length and the first lane of each live model's runs
  if (wave == 0) {
    const int c0 = lane < M && sm.mx[lane] > -HUGE_VAL ? sm.cnt[lane] : 0;
    const int c1 = lane + kWave < M && sm.mx[lane + kWave] > -HUGE_VAL ? sm.cnt[lane + kWave] : 0;
    int R = 1;
    for (; R < (LARGE ? NMAX : kRunMax); ++R) {
      int tot = (c0 + R - 1) / R + (c1 + R - 1) / R;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) tot += __shfl_xor(tot, o);
      if (tot <= kRwThreads) break;
    }
    const int r0 = (c0 + R - 1) / R, r1 = (c1 + R - 1) / R;
    const int i0 = wave_scan_incl(r0);
    const int i1 = wave_scan_incl(r1) + __shfl(i0, kWave - 1);
    if (lane < M) sm.rb[lane] = i0 - r0;
    if (lane + kWave < M) sm.rb[lane + kWave] = i1 - r1;
    if (lane == kWave - 1) sm.rb[M] = i1;
    if (lane == 0) sm.run_len = R;
  }
  __syncthreads();
  constexpr int RM = KIND == 0 ? 1 : (KIND == 1 ? kRunMax : 0);   // 0: runs read from LDS
  const RunLane run = run_of_lane<RM != 0>(sm, M);
  // temperature increment
  const double target = a.alpha_tess * (double)N;
  const double hi = 1.0 - g0;
  bool full;
  const double dg = next_increment<RM>(sm, run, hi, target, M, full);
  if (!full) {
    const double chosen[1] = {dg};
    double t1[1], unused;
    eval_tess<1, RM, false>(sm, run, chosen, t1, unused, M, true);   // s1 at the chosen increment
  }
  // evidence, quantised weights and per-model cumulative sums (wave per model)
  for (int m = wave; m < M; m += kRwWaves) {
    const int n = sm.cnt[m];
    if (n == 0) {
      // empty sum of incremental weights: the model's evidence estimate becomes 0
      if (lane == 0) log_z[(int64_t)s * M + m] = -HUGE_VAL;
      continue;
    }
    const double mx = sm.mx[m];
    const bool live = mx > -HUGE_VAL;
    const double inv = live ? 1.0 / sm.s1[m] : 0.0;
    if (lane == 0) {
      double &lz = log_z[(int64_t)s * M + m];
      lz = live ? lz + dg * mx + log(sm.s1[m]) - log((double)n) : -HUGE_VAL;
    }
    uint64_t carry = 0;
    for (int q0 = 0; q0 < n; q0 += kWave) {
      const int q = q0 + lane;
      uint64_t v = 0;
      if (q < n && live) {
        const double w = exp_tab(dg * xs[sm.base[m] + q], sm.e2) * inv;
        v = (uint64_t)rint(w * 0x1.0p60);
      }
      // inclusive scan over the wave
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const uint64_t t = __shfl_up(v, o);
        if (lane >= o) v += t;
      }
      if (q < n) sm.u.cum[sm.base[m] + q] = carry + v;
      carry += __shfl(v, kWave - 1);
    }
  }
  __syncthreads();
  // ancestors: member j of model m takes the first member whose cumulative weight
  // exceeds the j-th systematic threshold
  for (int i = tid; i < N; i += kRwThreads) sm.v.anc_l[i] = (int16_t)i;
  __syncthreads();
  for (int pos = tid; pos < N; pos += kRwThreads) {
    const int dest = sm.idx[pos];
    if (dest < 0 || dest >= N) {       // cannot happen for a complete sort; never write outside
      atomicOr(flags, kFlagUnsorted);
      continue;
    }
    const int m = sm.mod[dest];
    const int b = sm.base[m], n = sm.cnt[m];
    const uint64_t T = sm.u.cum[b + n - 1];
    int src = dest;
    if (T > 0) {
      const uint64_t thr = sys_threshold((uint64_t)(pos - b), sm.U[m], T, (uint64_t)n);
      int lo = 0, hi2 = n - 1;       // first q with cum[q] > thr (exists: cum[n-1] = T > thr)
      while (lo < hi2) {
        const int mid = (lo + hi2) >> 1;
        if (sm.u.cum[b + mid] > thr)
          hi2 = mid;
        else
          lo = mid + 1;
      }
      src = sm.idx[b + lo];
      if (src < 0 || src >= N) src = dest;
    }
    sm.v.anc_l[dest] = (int16_t)src;
  }
  __syncthreads();
  // the resampled population, in particle order (coalesced writes)
  for (int first = 0; first < N; first += kCP * kRwThreads)
    copy_resampled<kCP, kRB>(sm, in, ll_in, out, ll_out, anc, off, N, rows_c, rows_m, rows_zm, first);
  if (tid == 0) {
    gamma[s] = full ? 1.0 : g0 + dg;
    if (active) active[s] = 1;
  }
}

hipError_t launch_reweight_resample(const SmcShape &sh, const rjsmc_reweight_args &a, const DevParticles &in,
                                    const double *ll_in, const DevParticlesW &out, double *ll_out, double *gamma,
                                    double *log_z, int32_t *active, int32_t *anc, int *flags, const double *exp2t,
                                    hipStream_t stream) {
  const int64_t nps = in.n_per_sounding > 0 ? in.n_per_sounding : in.n;
  if (nps > kMaxPerSoundingLarge || sh.n_models > kMaxModels) return hipErrorInvalidValue;
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3((unsigned)a.n_sound), dim3(kRwThreads), 0, stream, sh, a, in, ll_in, out, ll_out,
                       gamma, log_z, active, anc, flags, exp2t);
  };
  if (nps <= kRwThreads)
    go(reweight_resample_kernel<0>);
  else if (nps <= kMaxPerSounding)
    go(reweight_resample_kernel<1>);
  else
    go(reweight_resample_kernel<2>);
  return hipGetLastError();
}

// ---------------------------------------------------------------- parameter vectors --
// theta = (phi_b, phi_1..k, z_1..k, m_1..l, zm_1..l, log10 tau, c) of a decoupled particle.
__host__ __device__ __forceinline__ DevParticles readonly(const DevParticlesW &w) {
  DevParticles r;
  r.n = w.n;
  r.stride = w.stride;
  r.n_per_sounding = w.n_per_sounding;
  r.layout = w.layout;
  r.kappa = w.kappa;
  r.lambda = w.lambda;
  r.phi_b = w.phi_b;
  r.phi = w.phi;
  r.z_cond = w.z_cond;
  r.m = w.m;
  r.z_charg = w.z_charg;
  r.log10_tau = w.log10_tau;
  r.c = w.c;
  return r;
}

__device__ __forceinline__ double theta_get(const DevParticles &p, int64_t i, int k, int l, int a) {
  const int64_t S = p.stride;
  if (a == 0) return p.phi_b[i];
  a -= 1;
  if (a < k) return p.phi[a * S + i];
  a -= k;
  if (a < k) return p.z_cond[a * S + i];
  a -= k;
  if (a < l) return p.m[a * S + i];
  a -= l;
  if (a < l) return p.z_charg[a * S + i];
  a -= l;
  return a == 0 ? p.log10_tau[i] : p.c[i];
}

__device__ __forceinline__ double prior_sd(const rjsmc_prior &pr, double zmax, int k, int l, int a) {
  const double r12 = 0.28867513459481288225;   // 1/sqrt(12)
  if (a <= k) return (pr.phi_hi - pr.phi_lo) * r12;
  if (a <= 2 * k) return zmax * r12;
  if (a <= 2 * k + l) return (pr.m_hi - pr.m_lo) * r12;
  if (a <= 2 * k + 2 * l) return zmax * r12;
  return a == 2 * k + 2 * l + 1 ? (pr.ltau_hi - pr.ltau_lo) * r12 : (pr.c_hi - pr.c_lo) * r12;
}

// ---------------------------------------------------------------------- adaptation ---
// One workgroup per (sounding, model): the member list (first wave, by ballot), the mean
// (a thread per component) and covariance (a thread per entry), each summed over the
// members in index order, then the factor of the covariance (eigen_factor).  (Starting
// the sweeps from the previous step's directions was tried: resampling leaves duplicate
// members, so those factors often have null directions, and where they did not the
// sweep count hardly fell.)
constexpr int kDimMax = 3 + 2 * (kMaxLayers - 1);   // 33
constexpr int kLd = kDimMax + 1;                    // LDS row stride
constexpr int kAdaptThreads = 512;                 // workgroup of the adaptation kernels

// Jacobi eigen-decomposition of the symmetric d x d matrix A (LDS, overwritten; V0 holds
// the identity, T two spare d x d buffers) and the factor F = U diag(sqrt Lambda) into
// F[r D + a] (direction r), eigenvalues descending, each direction signed so that its
// largest-magnitude component is positive.
//
// The sweeps use the round-robin (tournament) ordering: a sweep is nn - 1 rounds of nn/2
// disjoint index pairs (nn = d rounded up to even, the padding index nn - 1 when d is
// odd): in round r index nn - 1 meets r and every other index i meets (2r - i) mod
// (nn - 1).  Every pair of a round is rotated at once, A <- J^T A J with J the product of
// the round's rotations, together with V <- V J; each pair's 2x2 block is touched by its
// own rotation only, so its diagonal takes the classical update and its off-diagonal
// entry is set to zero.  A round is one pass and one barrier (the matrices ping-pong
// between two buffers), pipelined: waves 1.. apply round r's rotations (read from a
// two-slot table) to the strictly upper entries of A (mirrored) and to V, while lane i
// of wave 0 owns index i: it keeps i's rotation and new diagonal in registers, writes
// that diagonal, and forms the rotation of i's pair in round r + 1 from the pair's 2x2
// block after round r (its partner's state by lane exchange, the off-diagonal entry by
// the same expression as the other waves), so that both lanes of a pair derive the same
// rotation.  The rotations of the first round are formed before the sweeps.
__device__ __forceinline__ double jacobi_entry(double cx, double sx, double cj, double sj, double axj, double axy,
                                               double ayj, double ayy) {
  // entry (x, j) of J^T A J: cx (cj a_xj + sj a_x,yj) + sx (cj a_yx,j + sj a_yx,yj), fused
  // the same way wherever it is evaluated
  return fma(cx, fma(cj, axj, sj * axy), sx * fma(cj, ayj, sj * ayy));
}

// 1/sqrt(x) for finite normal x > 0: the hardware estimate y and one third-order step,
// y (1 - v)^(-1/2) ~ y (1 + v/2 + 3v^2/8) with v = 1 - x y^2 (remainder below 2^-70).
__device__ __forceinline__ double rsqrt_fast(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double v = fma(-(x * y), y, 1.0);
  return fma(y * v, fma(v, 0.375, 0.5), y);
}

// Rotation of the pair (p, q), p < q, from its 2x2 block: c, s with J[p][p] = J[q][q] = c,
// J[p][q] = s = -J[q][p], and the rotated diagonal entries (identity if apq = 0).  The
// angle phi is the smaller solution, t = tan phi the smaller root of t^2 + 2 theta t - 1 = 0
// with theta = (aqq - app) / (2 apq).  With rho = 1 / sqrt((aqq - app)^2 + 4 apq^2),
// cos 2phi = |aqq - app| rho and h = cos^2 phi = (1 + cos 2phi) / 2 lies in [1/2, 1], so
// with q = 1 / sqrt(h): c = h q, |s| = |t| c = |apq| rho q (h q^2 = 1), and
// |t apq| = apq^2 rho q^2, the sign of t being that of (aqq - app) apq (two reciprocal
// square roots, no division; after q, one product for c and s and a product and a fused
// multiply-add for the diagonal: the chain that bounds a round).
__device__ __forceinline__ void jacobi_rotation(double app, double aqq, double apq, double &c, double &s,
                                                double &dp, double &dq) {
  c = 1.0;
  s = 0.0;
  dp = app;
  dq = aqq;
  if (apq == 0.0) return;
  const double dd = aqq - app;
  const double rho = rsqrt_fast(fma(dd, dd, 4.0 * apq * apq));
  const double h = fma(0.5 * fabs(dd), rho, 0.5);
  const double q = rsqrt_fast(h);
  const double ar = fabs(apq) * rho;
  const double w = dd >= 0.0 ? -(fabs(apq) * ar) : fabs(apq) * ar;   // -t apq / q^2
  const double q2 = q * q;
  c = h * q;
  s = (dd >= 0.0) == (apq >= 0.0) ? ar * q : -(ar * q);
  dp = fma(w, q2, app);
  dq = fma(-w, q2, aqq);
}

template <int NT>
__device__ __forceinline__ void eigen_factor(double (*A)[kLd], double (*V0)[kLd], double (*T)[kDimMax][kLd],
                                             int *order, int d, int D, double *F) {
  static_assert(NT >= 2 * kWave, "the pipelined rounds need wave 0 and at least one more wave");
  static_assert(kDimMax <= kWave, "wave 0 holds one index per lane");
  constexpr int kBulk = NT - kWave;             // threads of waves 1..
  constexpr int kItems = (kDimMax * (kDimMax - 1) / 2 + kDimMax * kDimMax + kBulk - 1) / kBulk;
  constexpr int NW = NT / kWave;
  const int tid = threadIdx.x;
  __shared__ double red[2][2][NW];              // per sweep parity: the waves' off-diagonal and diagonal sums
  __shared__ double2 rot_cs[2][kDimMax + 1];    // per index i of a round: (J[i][i], J[partner][i]); slot kDimMax: (1, 0)
  double (*Ac)[kLd] = A;         // current matrix and eigenvector estimate, and the
  double (*An)[kLd] = T[0];      // buffers a round writes (swapped after each round)
  double (*Vc)[kLd] = V0;
  double (*Vn)[kLd] = T[1];
  const int nn = (d + 1) & ~1, nr = nn - 1;
  // partner of index i in round r; an index paired with the padding index is its own
  auto partner = [nr, d](int i, int r) {
    int y = 2 * r - i;
    y += y < 0 ? nr : 0;
    y -= y >= nr ? nr : 0;
    y = i == r ? nr : y;
    y = i == nr ? r : y;
    return y < d ? y : i;
  };
  // the waves' sums of squares of the off-diagonal and diagonal entries, added in wave
  // order (all threads; slot `sl` of red, one barrier)
  auto converged = [&](double offn, double diag, int sl) {
    offn = wave_sum(offn);
    diag = wave_sum(diag);
    if ((tid & (kWave - 1)) == 0) {
      red[sl][0][tid / kWave] = offn;
      red[sl][1][tid / kWave] = diag;
    }
    __syncthreads();
    offn = 0.0;
    diag = 0.0;
    for (int w = 0; w < NW; ++w) {
      offn += red[sl][0][w];
      diag += red[sl][1][w];
    }
    return !(offn > 1e-24 * diag);
  };
  // the bulk threads' items: strictly upper entries of A, then the entries of V
  const int nA = d * (d - 1) / 2, nItems = nA + d * d;
  int ix[kItems], ij[kItems];
#pragma unroll
  for (int e = 0; e < kItems; ++e) {
    int t = tid - kWave + e * kBulk;
    ix[e] = -1;
    ij[e] = 0;
    if (tid < kWave || t >= nItems) continue;
    if (t < nA) {
      int a = 0;
      while (t >= d - 1 - a) {         // row a of the strict upper triangle holds d - 1 - a entries
        t -= d - 1 - a;
        ++a;
      }
      ix[e] = a;
      ij[e] = a + 1 + t;
    } else {
      t -= nA;
      ix[e] = kDimMax + t / d;         // V entry, row offset by kDimMax
      ij[e] = t % d;
    }
  }
  // wave 0, lane i: index i's rotation (c, s) and its diagonal after the round in progress
  // (a pair that is not rotated has s = 0)
  double my_c = 1.0, my_s = 0.0, my_dn = 0.0;
  double offn = 0.0, diag = 0.0;
  if (tid < d) {
    const int y = partner(tid, 0);
    my_dn = Ac[tid][tid];
    diag = my_dn * my_dn;
    if (y != tid) {
      const int p = min(tid, y), q = max(tid, y);
      double c, sn, dp, dq;
      jacobi_rotation(Ac[p][p], Ac[q][q], Ac[p][q], c, sn, dp, dq);
      my_c = c;
      my_s = tid == p ? -sn : sn;
      my_dn = tid == p ? dp : dq;
    }
    rot_cs[0][tid] = make_double2(my_c, my_s);
  }
  if (tid < 2) rot_cs[tid][kDimMax] = make_double2(1.0, 0.0);   // the identity, for the rows of V
#pragma unroll
  for (int e = 0; e < kItems; ++e)
    if (ix[e] >= 0 && ix[e] < kDimMax) offn += 2.0 * Ac[ix[e]][ij[e]] * Ac[ix[e]][ij[e]];
  bool done = converged(offn, diag, 1);
  int g = 0;                           // rounds done (table slot of the next round: g & 1)
  for (int sweep = 0; sweep < 40 && !done; ++sweep) {
    for (int round = 0; round < nr; ++round, ++g) {
      const int sl = g & 1;
      const bool last = round + 1 == nr; // this round's result is tested for convergence
      offn = 0.0;
      diag = 0.0;
      if (tid < kWave) {
        // the partner in the next round, the 2x2 block's entries before this round (all
        // loads ahead of this round's stores), and the partner's state in this round by
        // lane exchange (every lane of the wave takes part)
        const int r1 = last ? 0 : round + 1;
        const int i = tid < d ? tid : 0;
        const int y1 = partner(i, r1);
        const bool low = i < y1;
        const int p = low ? i : y1, q = low ? y1 : i;
        const int yp = partner(p, round), yq = partner(q, round);
        const double m0 = Ac[p][q], m1 = Ac[p][yq], m2 = Ac[yp][q], m3 = Ac[yp][yq];
        const double c_y = __shfl(my_c, y1), s_y = __shfl(my_s, y1), dn_y = __shfl(my_dn, y1);
        if (tid < d) {
          const double dn_now = my_dn;
          double c = 1.0, sn = 0.0, dp = my_dn, dq = my_dn;
          if (y1 != i) {
            const double cp = low ? my_c : c_y, sp = low ? my_s : s_y;
            const double cq = low ? c_y : my_c, sq = low ? s_y : my_s;
            double apq = jacobi_entry(cp, sp, cq, sq, m0, m1, m2, m3);
            apq = q == yp ? 0.0 : apq;   // (p, q) rotated in this round as well (only when nn = 2)
            jacobi_rotation(low ? my_dn : dn_y, low ? dn_y : my_dn, apq, c, sn, dp, dq);
          }
          my_c = c;
          my_s = low ? -sn : sn;
          my_dn = low ? dp : dq;
          An[i][i] = dn_now;
          diag = dn_now * dn_now;
          rot_cs[sl ^ 1][i] = make_double2(my_c, my_s);
        }
      } else {
        // all loads of the thread's items, then the entries and the stores; a V entry is
        // the same expression with the identity for its row (table slot kDimMax)
        double2 lx[kItems], lj[kItems];
        double m0[kItems], m1[kItems], m2[kItems], m3[kItems];
#pragma unroll
        for (int e = 0; e < kItems; ++e) {
          const int x = ix[e], j = ij[e];
          if (x < 0) continue;
          const bool isA = x < kDimMax;
          const int r = isA ? x : x - kDimMax;
          const int yj = partner(j, round), yx = isA ? partner(x, round) : r;
          double (*M)[kLd] = isA ? Ac : Vc;
          lx[e] = rot_cs[sl][isA ? x : kDimMax];
          lj[e] = rot_cs[sl][j];
          m0[e] = M[r][j];
          m1[e] = M[r][yj];
          m2[e] = M[yx][j];
          m3[e] = M[yx][yj];
        }
#pragma unroll
        for (int e = 0; e < kItems; ++e) {
          const int x = ix[e], j = ij[e];
          if (x < 0) continue;
          const double v = jacobi_entry(lx[e].x, lx[e].y, lj[e].x, lj[e].y, m0[e], m1[e], m2[e], m3[e]);
          if (x < kDimMax) {           // A entry (x < j), mirrored; a pair of this round: 0
            const double a = j == partner(x, round) ? 0.0 : v;
            An[x][j] = a;
            An[j][x] = a;
            offn += 2.0 * a * a;
          } else {                     // V entry (x - kDimMax, j)
            Vn[x - kDimMax][j] = v;
          }
        }
      }
      if (last)
        done = converged(offn, diag, sweep & 1);   // (its barrier ends the round)
      else
        __syncthreads();
      double (*sw)[kLd] = Ac;
      Ac = An;
      An = sw;
      sw = Vc;
      Vc = Vn;
      Vn = sw;
    }
  }
  // descending eigenvalue order (stable selection by one thread)
  if (tid == 0) {
    for (int a = 0; a < d; ++a) order[a] = a;
    for (int a = 1; a < d; ++a) {
      const int v = order[a];
      int b = a;
      while (b > 0 && Ac[order[b - 1]][order[b - 1]] < Ac[v][v]) {
        order[b] = order[b - 1];
        --b;
      }
      order[b] = v;
    }
  }
  __syncthreads();
  // eigenvalues below 1e-12 of the largest are the rounding noise of a singular
  // covariance (a re-sampled model with fewer distinct members than dimensions): zero
  const double lmax = Ac[order[0]][order[0]];
  for (int r = tid; r < d; r += NT) {
    const int c = order[r];
    const double lc = Ac[c][c];
    const double ev = (lc > 0.0 && lc > 1e-12 * lmax) ? sqrt(lc) : 0.0;
    int big = 0;
    for (int a = 1; a < d; ++a)
      if (fabs(Vc[a][c]) > fabs(Vc[big][c])) big = a;
    const double sg = Vc[big][c] < 0.0 ? -1.0 : 1.0;
    for (int a = 0; a < d; ++a) F[r * D + a] = sg * ev * Vc[a][c];
  }
}

// Members of model (k, l) in sounding `off`, in index order, into mem; returns their
// count (all threads).  Each wave ballots a contiguous range of 64-particle chunks, the
// waves' counts are summed in wave order, then each wave places its members.
__device__ __forceinline__ int model_members(const DevParticles &p, int64_t off, int N, int k, int l,
                                             int16_t *mem, int *wcount) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  constexpr int NW = kAdaptThreads / kWave;
  const int n_chunks = (N + kWave - 1) / kWave, cpw = (n_chunks + NW - 1) / NW;
  const int ch0 = wave * cpw, ch1 = min(n_chunks, ch0 + cpw);
  int cnt = 0;
  for (int ch = ch0; ch < ch1; ++ch) {
    const int i = ch * kWave + lane;
    cnt += __popcll(__ballot(i < N && p.kappa[off + i] == k && p.lambda[off + i] == l));
  }
  if (lane == 0) wcount[wave] = cnt;
  __syncthreads();
  int base = 0, total = 0;
  for (int w = 0; w < NW; ++w) {
    base += w < wave ? wcount[w] : 0;
    total += wcount[w];
  }
  for (int ch = ch0; ch < ch1; ++ch) {
    const int i = ch * kWave + lane;
    const bool sel = i < N && p.kappa[off + i] == k && p.lambda[off + i] == l;
    const uint64_t bl = __ballot(sel);
    if (sel) mem[base + __popcll(bl & ((1ull << lane) - 1))] = (int16_t)i;
    base += __popcll(bl);
  }
  __syncthreads();
  return total;
}

// Moments and factor of one (sounding, model).  The members' parameter vectors are staged
// in LDS a chunk at a time by all threads (the chunk buffer is the eigen-solver's matrix
// storage, unused until then), the mean (a thread per component) and the covariance (a
// thread per upper-triangle entry) are summed over the members in index order, and the
// workgroup runs the Jacobi sweeps.
__global__ __launch_bounds__(kAdaptThreads) void adapt_kernel(SmcShape sh, DevParticles p, rjsmc_prior pr, double *factors) {
  __shared__ int16_t mem[kMaxPerSoundingLarge];
  __shared__ double AVT[4][kDimMax][kLd];    // A, V0, T[2] of the eigen solver; first the staged chunks
  __shared__ double mu[kDimMax];
  __shared__ int wcount[kAdaptThreads / kWave];
  __shared__ int order[kDimMax];
  double (*A)[kLd] = AVT[0];
  double (*V0)[kLd] = AVT[1];
  double (*T)[kDimMax][kLd] = AVT + 2;
  double *stage = &AVT[0][0][0];
  constexpr int kStage = 4 * kDimMax * kLd;
  const int tid = threadIdx.x;
  const int M = sh.n_models;
  const int s = blockIdx.x / M, m = blockIdx.x % M;
  const int N = (int)(p.n_per_sounding > 0 ? p.n_per_sounding : p.n);
  const int64_t off = (int64_t)s * N;
  const int k = m / (sh.km + 1), l = m % (sh.km + 1);
  const int d = 3 + 2 * k + 2 * l, D = sh.dmax;
  double *F = factors + (int64_t)blockIdx.x * D * D;
  const int nm = model_members(p, off, N, k, l, mem, wcount);
  const bool fallback = nm <= d;
  // the factor is rewritten whole: zero, or the fallback's prior-scaled diagonal
  for (int t = tid; t < D * D; t += kAdaptThreads) {
    const int a = t / D;
    F[t] = fallback && a < d && t == a * D + a ? 0.1 * prior_sd(pr, sh.z_max, k, l, a) : 0.0;
  }
  if (fallback) return;
  const int C = kStage / d;                    // members per staged chunk
  auto stage_chunk = [&](int q0, int nq) {     // stage[q * d + a] = theta_a of member q0 + q
    for (int t = tid; t < nq * d; t += kAdaptThreads) {
      const int q = t / d, a = t - q * d;
      stage[t] = theta_get(p, off + mem[q0 + q], k, l, a);
    }
  };
  // mean (a thread per component, members in index order)
  double acc_m = 0.0;
  for (int q0 = 0; q0 < nm; q0 += C) {
    const int nq = min(C, nm - q0);
    __syncthreads();
    stage_chunk(q0, nq);
    __syncthreads();
    if (tid < d)
      for (int q = 0; q < nq; ++q) acc_m += stage[q * d + tid];
  }
  if (tid < d) mu[tid] = acc_m / (double)nm;
  __syncthreads();
  // covariance (a thread per upper-triangle entry, members in index order); one staged
  // chunk when the members fit, else the chunks again
  const int ne = d * (d + 1) / 2;
  int ea[2] = {0, 0}, eb[2] = {0, 0};
  double acc_c[2] = {0.0, 0.0};
  for (int r = 0; r < 2; ++r) {
    int t = tid + r * kAdaptThreads, a = 0;
    if (t < ne) {
      while (t >= d - a) {                     // row a of the upper triangle holds d - a entries
        t -= d - a;
        ++a;
      }
      ea[r] = a;
      eb[r] = a + t;
    }
  }
  for (int q0 = 0; q0 < nm; q0 += C) {
    const int nq = min(C, nm - q0);
    if (q0 > 0 || nm > C) {                    // (a single chunk is still staged from the mean)
      __syncthreads();
      stage_chunk(q0, nq);
      __syncthreads();
    }
    for (int r = 0; r < 2; ++r) {
      if (tid + r * kAdaptThreads >= ne) continue;
      const int a = ea[r], b = eb[r];
      const double ma = mu[a], mb = mu[b];
      double acc = acc_c[r];
      for (int q = 0; q < nq; ++q) acc += (stage[q * d + a] - ma) * (stage[q * d + b] - mb);
      acc_c[r] = acc;
    }
  }
  __syncthreads();                             // the staged chunk is no longer read
  for (int r = 0; r < 2; ++r) {
    if (tid + r * kAdaptThreads >= ne) continue;
    const int a = ea[r], b = eb[r];
    A[a][b] = acc_c[r] / (double)(nm - 1);
    A[b][a] = A[a][b];
  }
  for (int t = tid; t < d * d; t += kAdaptThreads) V0[t / d][t % d] = t / d == t % d ? 1.0 : 0.0;
  __syncthreads();
  eigen_factor<kAdaptThreads>(A, V0, T, order, d, D, F);
}

hipError_t launch_adapt(const SmcShape &sh, const DevParticles &p, int n_sound, const rjsmc_prior &pr,
                        double *factors, hipStream_t stream) {
  hipLaunchKernelGGL(adapt_kernel, dim3((unsigned)(n_sound * sh.n_models)), dim3(kAdaptThreads), 0, stream, sh, p,
                     pr, factors);
  return hipGetLastError();
}

// ------------------------------------------------------------- particle recycling ---
// One wavefront per (sounding, model) pools the model's members of the current
// population and of the archive's used slots, weighted by the deterministic mixture of
// the sources (Section 3.2.4):
//   log nu = gamma_t ll - log sum_c exp(log N_c - log Z_c + gamma_c ll)
// over the sources c with N_c > 0 members and a finite log Z_c (L^0 = 1).  Four passes
// over the sources (member list rebuilt per source): counts, the largest log nu, the
// weight sums and weighted mean, the weighted covariance; then eigen_factor.
__global__ __launch_bounds__(kAdaptThreads) void adapt_recycled_kernel(SmcShape sh, DevParticles p, const double *ll,
                                                               const double *gamma, const double *log_z,
                                                               ArchiveView ar, rjsmc_prior pr, double *factors) {
  __shared__ int16_t mem[kMaxPerSoundingLarge];
  __shared__ double A[kDimMax][kLd];
  __shared__ double V0[kDimMax][kLd];
  __shared__ double T[2][kDimMax][kLd];
  __shared__ double mu[kDimMax];
  __shared__ int s_ready;
  __shared__ int order[kDimMax];
  __shared__ double wst[kWave];
  __shared__ double comp_lc[kMaxArchive + 1], comp_g[kMaxArchive + 1];
  double (*X)[kLd] = reinterpret_cast<double (*)[kLd]>(&T[0][0][0]);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int M = sh.n_models;
  const int n_sound = (int)(gridDim.x / M);
  const int s = blockIdx.x / M, m = blockIdx.x % M;
  const int N = (int)(p.n_per_sounding > 0 ? p.n_per_sounding : p.n);
  const int64_t n_total = p.n;
  const int k = m / (sh.km + 1), l = m % (sh.km + 1);
  const int d = 3 + 2 * k + 2 * l, D = sh.dmax;
  double *F = factors + (int64_t)blockIdx.x * D * D;
  const int Q = ar.n_used + 1;            // sources: archive slots 0 .. n_used - 1, then the current population
  const double g_t = gamma[s];
  // weights, mean and covariance on the first wave; the workgroup then decomposes
  auto moments = [&]() -> bool {
    // member list of source q (particle offsets within that source's sounding s)
    auto members = [&](int q) {
      const DevParticles &P = q < ar.n_used ? ar.pop : p;
      const int64_t off = (q < ar.n_used ? (int64_t)q * n_total : 0) + (int64_t)s * N;
      int nm = 0;
      for (int c0 = 0; c0 < N; c0 += kWave) {
        const int i = c0 + lane;
        const bool sel = i < N && P.kappa[off + i] == k && P.lambda[off + i] == l;
        const uint64_t b = __ballot(sel);
        if (sel) mem[nm + __popcll(b & ((1ull << lane) - 1))] = (int16_t)i;
        nm += __popcll(b);
      }
      wave_lds_sync();
      return nm;
    };
    auto src_ll = [&](int q, int i) {
      return q < ar.n_used ? ar.ll[(int64_t)q * n_total + (int64_t)s * N + i] : ll[(int64_t)s * N + i];
    };
    // 1. mixture components
    int nc = 0;
    for (int q = 0; q < Q; ++q) {
      const int nm = members(q);
      const double gq = q < ar.n_used ? ar.gamma[(int64_t)q * n_sound + s] : g_t;
      const double lz = q < ar.n_used ? ar.log_z[((int64_t)q * n_sound + s) * M + m] : log_z[(int64_t)s * M + m];
      if (nm > 0 && lz > -HUGE_VAL && lz < HUGE_VAL) {
        if (lane == 0) {
          comp_lc[nc] = log((double)nm) - lz;
          comp_g[nc] = gq;
        }
        ++nc;
      }
      wave_lds_sync();
    }
    auto log_nu = [&](double x) {
      const double num = g_t == 0.0 ? 0.0 : g_t * x;
      double mx = -HUGE_VAL;
      for (int c = 0; c < nc; ++c) mx = fmax(mx, comp_lc[c] + (comp_g[c] == 0.0 ? 0.0 : comp_g[c] * x));
      if (!(num > -HUGE_VAL) || !(mx > -HUGE_VAL)) return -HUGE_VAL;   // L = 0: weight 0
      double sum = 0.0;
      for (int c = 0; c < nc; ++c) sum += exp(comp_lc[c] + (comp_g[c] == 0.0 ? 0.0 : comp_g[c] * x) - mx);
      return num - (mx + log(sum));
    };
    // 2. largest log weight
    double lmax = -HUGE_VAL;
    for (int q = 0; q < Q; ++q) {
      const int nm = members(q);
      for (int r = lane; r < nm; r += kWave) lmax = fmax(lmax, log_nu(src_ll(q, mem[r])));
      wave_lds_sync();
    }
    lmax = wave_max(lmax);
    for (int t = lane; t < D * D; t += kWave) F[t] = 0.0;
    // 3. weight sums and weighted mean: members staged 64 at a time, lane a adds in order
    double acc_mu = 0.0, sw = 0.0, sw2 = 0.0;
    if (lmax > -HUGE_VAL) {
      for (int q = 0; q < Q; ++q) {
        const int nm = members(q);
        const DevParticles &P = q < ar.n_used ? ar.pop : p;
        const int64_t off = (q < ar.n_used ? (int64_t)q * n_total : 0) + (int64_t)s * N;
        for (int q0 = 0; q0 < nm; q0 += kWave) {
          const int r = q0 + lane;
          if (r < nm) {
            const double w = exp(log_nu(src_ll(q, mem[r])) - lmax);
            wst[lane] = w;
            sw += w;
            sw2 += w * w;
            for (int a = 0; a < d; ++a) X[lane][a] = theta_get(P, off + mem[r], k, l, a);
          }
          wave_lds_sync();
          const int nq = nm - q0 < kWave ? nm - q0 : kWave;
          if (lane < d)
            for (int rr = 0; rr < nq; ++rr) acc_mu += wst[rr] * X[rr][lane];
          wave_lds_sync();
        }
      }
    }
    sw = wave_sum(sw);
    sw2 = wave_sum(sw2);
    if (!(lmax > -HUGE_VAL) || !(sw * sw > (double)d * sw2)) {      // effective sample size <= d
      for (int a = lane; a < d; a += kWave) F[a * D + a] = 0.1 * prior_sd(pr, sh.z_max, k, l, a);
      return false;
    }
    if (lane < d) mu[lane] = acc_mu / sw;
    for (int t = lane; t < d * d; t += kWave) A[t / d][t % d] = 0.0;
    wave_lds_sync();
    // 4. weighted covariance sum w (theta - mu)(theta - mu)^T, then / (sw - sw2 / sw)
    for (int q = 0; q < Q; ++q) {
      const int nm = members(q);
      const DevParticles &P = q < ar.n_used ? ar.pop : p;
      const int64_t off = (q < ar.n_used ? (int64_t)q * n_total : 0) + (int64_t)s * N;
      for (int q0 = 0; q0 < nm; q0 += kWave) {
        const int r = q0 + lane;
        if (r < nm) {
          wst[lane] = exp(log_nu(src_ll(q, mem[r])) - lmax);
          for (int a = 0; a < d; ++a) X[lane][a] = theta_get(P, off + mem[r], k, l, a) - mu[a];
        }
        wave_lds_sync();
        const int nq = nm - q0 < kWave ? nm - q0 : kWave;
        for (int t = lane; t < d * d; t += kWave) {
          const int a = t / d, b = t % d;
          if (b < a) continue;
          double acc = A[a][b];
          for (int rr = 0; rr < nq; ++rr) acc += wst[rr] * X[rr][a] * X[rr][b];
          A[a][b] = acc;
        }
        wave_lds_sync();
      }
    }
    const double norm = sw - sw2 / sw;      // sum w (1 - sum w~^2)
    for (int t = lane; t < d * d; t += kWave) {
      const int a = t / d, b = t % d;
      if (b >= a) A[a][b] = A[a][b] / norm;
    }
    wave_lds_sync();
    for (int t = lane; t < d * d; t += kWave) {
      const int a = t / d, b = t % d;
      if (b < a) A[a][b] = A[b][a];
      V0[a][b] = a == b ? 1.0 : 0.0;
    }
    wave_lds_sync();
    return true;
  };
  if (wave == 0) {
    const bool ok = moments();
    if (lane == 0) s_ready = ok ? 1 : 0;
  }
  __syncthreads();
  if (!s_ready) return;
  eigen_factor<kAdaptThreads>(A, V0, T, order, d, D, F);
}

hipError_t launch_adapt_recycled(const SmcShape &sh, const DevParticles &p, const double *ll, const double *gamma,
                                 const double *log_z, int n_sound, const ArchiveView &ar, const rjsmc_prior &pr,
                                 double *factors, hipStream_t stream) {
  hipLaunchKernelGGL(adapt_recycled_kernel, dim3((unsigned)(n_sound * sh.n_models)), dim3(kAdaptThreads), 0, stream,
                     sh, p, ll, gamma, log_z, ar, pr, factors);
  return hipGetLastError();
}

// Slot `slot` of the archive := population src (every row), its ll, gamma and log_z.
__global__ __launch_bounds__(256) void archive_store_kernel(DevParticles src, const double *ll, const double *gamma,
                                                            const double *log_z, int n_sound, int n_models,
                                                            DevParticlesW dst, double *ll_dst, double *gamma_dst,
                                                            double *log_z_dst, int slot, int rows_c, int rows_m,
                                                            int rows_zm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = src.n, Si = src.stride, So = dst.stride;
  const int64_t o = (int64_t)slot * n + i;
  if (i < n) {
    dst.kappa[o] = src.kappa[i];
    dst.lambda[o] = src.lambda[i];
    dst.phi_b[o] = src.phi_b[i];
    dst.log10_tau[o] = src.log10_tau[i];
    dst.c[o] = src.c[i];
    ll_dst[o] = ll[i];
    for (int r = 0; r < rows_c; ++r) {
      dst.phi[r * So + o] = src.phi[r * Si + i];
      dst.z_cond[r * So + o] = src.z_cond[r * Si + i];
    }
    for (int r = 0; r < rows_m; ++r) dst.m[r * So + o] = src.m[r * Si + i];
    for (int r = 0; r < rows_zm; ++r) dst.z_charg[r * So + o] = src.z_charg[r * Si + i];
  }
  if (i < n_sound) gamma_dst[(int64_t)slot * n_sound + i] = gamma[i];
  if (i < (int64_t)n_sound * n_models) log_z_dst[(int64_t)slot * n_sound * n_models + i] = log_z[i];
}

hipError_t launch_archive_store(const DevParticles &src, const double *ll, const double *gamma, const double *log_z,
                                int n_sound, int n_models, const DevParticlesW &dst, double *ll_dst, double *gamma_dst,
                                double *log_z_dst, int slot, int rows_c, int rows_m, int rows_zm, hipStream_t stream) {
  int64_t work = src.n;
  if ((int64_t)n_sound * n_models > work) work = (int64_t)n_sound * n_models;
  const int64_t blocks = (work + 255) / 256;
  hipLaunchKernelGGL(archive_store_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, src, ll, gamma, log_z, n_sound,
                     n_models, dst, ll_dst, gamma_dst, log_z_dst, slot, rows_c, rows_m, rows_zm);
  return hipGetLastError();
}

// ------------------------------------------------------------------------ mutation ---
__device__ __forceinline__ int draw_type(const rjsmc_mutate_args &a, double u0) {
  double cum[RJSMC_N_MOVES];
  double acc = 0.0;
  for (int t = 0; t < RJSMC_N_MOVES; ++t) {
    acc += a.move_prob[t];
    cum[t] = acc;
  }
  const double x = u0 * acc;
  for (int t = 0; t < RJSMC_N_MOVES; ++t)
    if (x < cum[t]) return t;
  return RJSMC_N_MOVES - 1;
}

__device__ __forceinline__ bool in_range(double v, double lo, double hi) { return v >= lo && v <= hi; }

// Move type of every particle for sweep `move` (-1: inactive sounding or counts outside
// the capacities); mask = 2 marks the particles that take a gradient-informed step and
// whose current gradient is not already up to date (gvalid) from an earlier sweep.
__global__ __launch_bounds__(256) void draw_types_kernel(rjsmc_mutate_args a, int move, DevParticles st, int kc,
                                                         int km, int32_t *mask, int32_t *type,
                                                         const int32_t *active, const int32_t *gvalid) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= st.n) return;
  const int64_t snd = st.n_per_sounding > 0 ? i / st.n_per_sounding : 0;
  const int k = st.kappa[i], l = st.lambda[i];
  int t = -1;
  if ((!active || active[snd]) && k >= 0 && k <= kc && l >= 0 && l <= km) {
    double u0, ua;
    uniforms(a.seed, (uint32_t)i, (uint32_t)step_of(a), (uint32_t)move, 0u, u0, ua);
    t = draw_type(a, u0);
  }
  type[i] = t;
  mask[i] = t == RJSMC_MOVE_WITHIN_MALA && !(gvalid && gvalid[i]) ? 2 : 0;
}

// theta' = theta + F (eps^2/2 F^T (gamma grad) + eps xi) of the preconditioned Langevin step,
// in parameter-vector order; xi from uniform slots 3, 4, ... (Box-Muller pairs).
__device__ __forceinline__ void mala_normals(const rjsmc_mutate_args &a, int64_t i, int move, int d, double *xi) {
  for (int r = 0; r < d; r += 2) {
    double u1, u2;
    uniforms(a.seed, (uint32_t)i, (uint32_t)step_of(a), (uint32_t)move, (uint32_t)(3 + r / 2), u1, u2);
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(6.283185307179586477 * u2, &sn, &cs);
    xi[r] = rad * cs;
    if (r + 1 < d) xi[r + 1] = rad * sn;
  }
}

// ------------------------------------------------------------ adaptive birth ---
// a - b c with the product rounded before the difference.
__device__ __forceinline__ double msub_rn(double a, double b, double c) {
#pragma clang fp contract(off)
  return a - b * c;
}

// Row i of the symmetric root S = sum_r f_r f_r^T / |f_r| of F F^T (F[a][r] = Fm[r D + a],
// the nonzero columns), the columns added in order with separately rounded products.
__device__ void zca_row(const double *Fm, int D, int d, int i, double *row) {
#pragma clang fp contract(off)
  for (int j = 0; j < d; ++j) row[j] = 0.0;
  for (int r = 0; r < d; ++r) {
    const double *col = Fm + (int64_t)r * D;
    double n2 = 0.0;
    for (int q = 0; q < d; ++q) n2 = n2 + col[q] * col[q];
    if (n2 > 0.0) {
      const double w = col[i] / sqrt(n2);
      for (int j = 0; j < d; ++j) row[j] = row[j] + w * col[j];
    }
  }
}

// Adaptive birth (Appendix E.2) of an interface at depth zn in partition `part` (0
// conductivity, 1 chargeability) of the parameter vector th of model (k, l), or the
// death of interface r, the inverse map with the same covariance root (that of the
// larger model).  th is rewritten in place (kDimMax + 2 entries); false when the
// proposal is rejected outright; lq receives the log proposal correction.
__device__ bool zca_move(double *th, int &k, int &l, bool birth, int part, double u1, double up,
                         const rjsmc_mutate_args &a, const SmcShape &sh, int64_t snd, double &lq) {
  const int D = sh.dmax;
  const rjsmc_prior &pr = a.prior;
  const double dv = part == 0 ? pr.phi_hi - pr.phi_lo : pr.m_hi - pr.m_lo;
  const double log_norm = 0.91893853320467274178;   // log sqrt(2 pi)
  double S[kDimMax + 2];
  if (birth) {
    const int d = 3 + 2 * k + 2 * l;
    const double zn = sh.z_max * u1;
    int r = 0, ia, ib;
    double src;
    if (part == 0) {
      while (r < k && th[1 + k + r] < zn) ++r;
      ia = r + 1;                      // the new property's component
      ib = 1 + k + r;                  // the new depth goes to ib + 1
      src = th[r];
    } else {
      const int mo = 1 + 2 * k, zo = 1 + 2 * k + l;
      while (r < l && th[zo + r] < zn) ++r;
      ia = mo + r;
      ib = zo + r;
      src = r >= 1 ? th[mo + r - 1] : 0.0;
    }
    for (int q = d - 1; q >= ib; --q) th[q + 2] = th[q];
    th[ib + 1] = zn;
    for (int q = ib - 1; q >= ia; --q) th[q + 1] = th[q];
    th[ia] = src;
    const int kb = part == 0 ? k + 1 : k, lb = part == 0 ? l : l + 1, db = d + 2;
    const int jn = ia, jz = ib + 1, js = (part == 0 || r >= 1) ? ia - 1 : -1;
    const double *Fm = a.factors + (snd * sh.n_models + kb * (sh.km + 1) + lb) * (int64_t)D * D;
    zca_row(Fm, D, db, jn, S);
    for (int j = 0; j < db; ++j)
      if (j != jz) th[j] = madd_rn(th[j], S[j], up);
    const double J = S[jn] - (js >= 0 ? S[js] : 0.0);
    if (J == 0.0) return false;
    lq = log(fabs(J)) - log(dv) + (0.5 * up * up + log_norm);
    k = kb;
    l = lb;
    return true;
  }
  const int n_if = part == 0 ? k : l;
  if (n_if < 1) return false;
  int r = (int)(u1 * (double)n_if);
  r = r > n_if - 1 ? n_if - 1 : r;
  const int d = 3 + 2 * k + 2 * l;
  const int jn = part == 0 ? r + 1 : 1 + 2 * k + r;
  const int js = part == 0 ? r : (r >= 1 ? jn - 1 : -1);
  const int jz = part == 0 ? 1 + k + r : 1 + 2 * k + l + r;
  const double *Fm = a.factors + (snd * sh.n_models + k * (sh.km + 1) + l) * (int64_t)D * D;
  zca_row(Fm, D, d, jn, S);
  const double J = S[jn] - (js >= 0 ? S[js] : 0.0);
  if (J == 0.0) return false;
  const double upd = (th[jn] - (js >= 0 ? th[js] : 0.0)) / J;
  const double ud = th[jz];
  for (int j = 0; j < d; ++j)
    if (j != jz) th[j] = msub_rn(th[j], S[j], upd);
  int w = jn;                          // drop components jn and jz (jn < jz)
  for (int q = jn + 1; q < d; ++q)
    if (q != jz) th[w++] = th[q];
  const int ks = part == 0 ? k - 1 : k, ls = part == 0 ? l : l - 1;
  const int z0 = part == 0 ? 1 + ks : 1 + 2 * ks + ls, nz = part == 0 ? ks : ls;
  int below = 0;
  for (int q = 0; q < nz; ++q) {
    if (th[z0 + q] == ud) return false;
    below += th[z0 + q] < ud ? 1 : 0;
  }
  if (below != r) return false;        // u_d would not be inserted at index r: no bijection
  lq = -(log(fabs(J)) - log(dv) + (0.5 * upd * upd + log_norm));
  k = ks;
  l = ls;
  return true;
}

// One thread's column of an LDS array laid out [entry][thread].
struct LdsColumn {
  double *p;
  int stride;
  __device__ double &operator[](int j) const { return p[(int64_t)j * stride]; }
};

// Rows [0, n) of two row-major particle arrays (row j of particle i at a[j S + i]) into
// two LDS columns.  The loads go out in batches of kRowBatch rows, before the batch's
// stores: the compiler cannot move a global load above an LDS store through a generic
// pointer, so a plain row loop would wait out one load latency per row.
constexpr int kRowBatch = 8;
__device__ __forceinline__ void load_rows2(const double *a, const double *b, int64_t S, int64_t i, int n,
                                           const LdsColumn &da, const LdsColumn &db) {
  for (int j0 = 0; j0 < n; j0 += kRowBatch) {
    double va[kRowBatch], vb[kRowBatch];
#pragma unroll
    for (int t = 0; t < kRowBatch; ++t) {
      va[t] = j0 + t < n ? a[(int64_t)(j0 + t) * S + i] : 0.0;
      vb[t] = j0 + t < n ? b[(int64_t)(j0 + t) * S + i] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < kRowBatch; ++t)
      if (j0 + t < n) {
        da[j0 + t] = va[t];
        db[j0 + t] = vb[t];
      }
  }
}

// x[j] += step fx[j] and y[j] += step fy[j] (madd_rn) for j < n over two LDS columns, the
// factor entries (global) loaded in batches before the updates.
__device__ __forceinline__ void madd_rows2(const LdsColumn &x, const LdsColumn &y, const double *fx, const double *fy,
                                           int n, double step) {
  for (int j0 = 0; j0 < n; j0 += kRowBatch) {
    double vx[kRowBatch], vy[kRowBatch];
#pragma unroll
    for (int t = 0; t < kRowBatch; ++t) {
      vx[t] = j0 + t < n ? fx[j0 + t] : 0.0;
      vy[t] = j0 + t < n ? fy[j0 + t] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < kRowBatch; ++t)
      if (j0 + t < n) {
        x[j0 + t] = madd_rn(x[j0 + t], step, vx[t]);
        y[j0 + t] = madd_rn(y[j0 + t], step, vy[t]);
      }
  }
}

// Rows [0, n) of two row-major arrays copied from (sa, sb; stride Ss) to (da, db; stride
// Sd) for particle i, loads batched before stores as above.
__device__ __forceinline__ void copy_rows2(double *da, double *db, int64_t Sd, const double *sa, const double *sb,
                                           int64_t Ss, int64_t i, int n) {
  for (int j0 = 0; j0 < n; j0 += kRowBatch) {
    double va[kRowBatch], vb[kRowBatch];
#pragma unroll
    for (int t = 0; t < kRowBatch; ++t) {
      va[t] = j0 + t < n ? sa[(int64_t)(j0 + t) * Ss + i] : 0.0;
      vb[t] = j0 + t < n ? sb[(int64_t)(j0 + t) * Ss + i] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < kRowBatch; ++t)
      if (j0 + t < n) {
        da[(int64_t)(j0 + t) * Sd + i] = va[t];
        db[(int64_t)(j0 + t) * Sd + i] = vb[t];
      }
  }
}

// Proposal of move `move` for every particle (type from draw_types_kernel): written to
// `prop`; mask[i] = 1 if the proposal needs a likelihood, 2 if it needs a likelihood and
// a gradient, 0 if it is rejected outright.  MALA / ZCA: whether the launch can hold
// gradient-informed moves / the adaptive birth (without them their branches, and the
// private arrays they need, are compiled out; a particle drawn for an excluded move is
// rejected).
// A particle's state held by the caller: counts and scalars in registers, layer rows
// already in the thread's LDS columns (the proposal's layout).
struct StateRegs {
  int k, l;
  double phb, lt, cc;
};

template <bool MALA, bool ZCA>
__device__ __forceinline__ void propose_particle(int64_t i, const SmcShape &sh, const rjsmc_mutate_args &a, int move,
                                                 const DevParticles &st, const DevParticlesW &prop, int32_t *mask,
                                                 int32_t *type, const double *gamma, const DevParticles &gcur,
                                                 int32_t *gvalid, double *lq, const int32_t *active, int draw,
                                                 const StateRegs *pre = nullptr) {
  if (i >= st.n) return;
  const int64_t snd = st.n_per_sounding > 0 ? i / st.n_per_sounding : 0;
  const int64_t S = st.stride, So = prop.stride;
  int t;
  if (draw) {                          // the move type, as draw_types_kernel (no gradient moves)
    const int k0 = pre ? pre->k : st.kappa[i], l0 = pre ? pre->l : st.lambda[i];
    int t0 = -1;
    if ((!active || active[snd]) && k0 >= 0 && k0 <= sh.kc && l0 >= 0 && l0 <= sh.km) {
      double u0, ua;
      uniforms(a.seed, (uint32_t)i, (uint32_t)step_of(a), (uint32_t)move, 0u, u0, ua);
      t0 = draw_type(a, u0);
    }
    type[i] = t0;
    t = t0;
  } else {
    t = type[i];
  }
  if (t < 0) {
    mask[i] = 0;
    return;
  }
  if (t == RJSMC_MOVE_WITHIN_MALA && gvalid) gvalid[i] = 1;   // computed just before, or kept
  const int kc = sh.kc, km = sh.km;
  const rjsmc_prior &pr = a.prior;
  double u1, u2, u3, u4;
  uniforms(a.seed, (uint32_t)i, (uint32_t)step_of(a), (uint32_t)move, 1u, u1, u2);
  uniforms(a.seed, (uint32_t)i, (uint32_t)step_of(a), (uint32_t)move, 2u, u3, u4);
  int k = pre ? pre->k : st.kappa[i], l = pre ? pre->l : st.lambda[i];
  // the layer arrays in LDS (one column per thread): private arrays indexed at run time
  // would live in scratch memory
  extern __shared__ double prop_lds[];
  const int T = blockDim.x;
  double *lds0 = prop_lds + threadIdx.x;
  const LdsColumn zc{lds0, T}, ph{lds0 + (int64_t)kc * T, T}, zm{lds0 + (int64_t)2 * kc * T, T},
      mm{lds0 + (int64_t)(2 * kc + km) * T, T};
  double phb, lt, cc;
  if (pre) {
    phb = pre->phb;
    lt = pre->lt;
    cc = pre->cc;
  } else {
    phb = st.phi_b[i];
    lt = st.log10_tau[i];
    cc = st.c[i];
    load_rows2(st.z_cond, st.phi, S, i, k, zc, ph);
    load_rows2(st.z_charg, st.m, S, i, l, zm, mm);
  }
  bool ok = false;
  const bool jump = t == RJSMC_MOVE_SIGMA_BIRTH || t == RJSMC_MOVE_M_BIRTH || t == RJSMC_MOVE_SIGMA_DEATH ||
                    t == RJSMC_MOVE_M_DEATH;
  // the standard normal of the moves that take one, formed once before the branches (a
  // wave runs the branches of all its lanes' move types one after another, and the
  // logarithm and cosine are its longest chain)
  const double nz = normal0(u2, u3);
  // the random-walk move's factor column and scale, requested before the branches (their
  // loads are in flight while the wave runs the other move types' branches)
  const double *Fr = nullptr;
  double rw_scale = 0.0, f0 = 0.0, fa = 0.0, fb = 0.0;
  if (t == RJSMC_MOVE_WITHIN_RW) {
    const int d = 3 + 2 * k + 2 * l;
    int r = (int)(u1 * (double)d);
    r = r > d - 1 ? d - 1 : r;
    const int mdl = k * (km + 1) + l;
    Fr = a.factors + ((snd * sh.n_models + mdl) * (int64_t)sh.dmax + r) * sh.dmax;
    rw_scale = a.rw_scale_dev ? a.rw_scale_dev[snd] : a.rw_scale;
    f0 = Fr[0];
    fa = Fr[d - 2];
    fb = Fr[d - 1];
  }
  if (lq) lq[i] = 0.0;
  if (ZCA && a.zca_birth && jump) {
    const bool birth = t == RJSMC_MOVE_SIGMA_BIRTH || t == RJSMC_MOVE_M_BIRTH;
    const int part = t == RJSMC_MOVE_SIGMA_BIRTH || t == RJSMC_MOVE_SIGMA_DEATH ? 0 : 1;
    if (!birth || (part == 0 ? k < kc : l < km)) {
      double th[kDimMax + 2], corr = 0.0;
      int q = 0;
      th[q++] = phb;
      for (int j = 0; j < k; ++j) th[q++] = ph[j];
      for (int j = 0; j < k; ++j) th[q++] = zc[j];
      for (int j = 0; j < l; ++j) th[q++] = mm[j];
      for (int j = 0; j < l; ++j) th[q++] = zm[j];
      th[q++] = lt;
      th[q++] = cc;
      if (zca_move(th, k, l, birth, part, u1, nz, a, sh, snd, corr)) {
        q = 0;
        phb = th[q++];
        for (int j = 0; j < k; ++j) ph[j] = th[q++];
        for (int j = 0; j < k; ++j) zc[j] = th[q++];
        for (int j = 0; j < l; ++j) mm[j] = th[q++];
        for (int j = 0; j < l; ++j) zm[j] = th[q++];
        lt = th[q++];
        cc = th[q++];
        ok = in_range(phb, pr.phi_lo, pr.phi_hi) && in_range(lt, pr.ltau_lo, pr.ltau_hi) &&
             in_range(cc, pr.c_lo, pr.c_hi);
        for (int j = 0; j < k; ++j)
          ok = ok && in_range(ph[j], pr.phi_lo, pr.phi_hi) && zc[j] > 0.0 && zc[j] < sh.z_max &&
               (j == 0 || zc[j] > zc[j - 1]);
        for (int j = 0; j < l; ++j)
          ok = ok && in_range(mm[j], pr.m_lo, pr.m_hi) && zm[j] > 0.0 && zm[j] < sh.z_max &&
               (j == 0 || zm[j] > zm[j - 1]);
        if (lq) lq[i] = corr;
      }
    }
  } else if (t == RJSMC_MOVE_SIGMA_BIRTH || t == RJSMC_MOVE_M_BIRTH) {
    const bool sig = t == RJSMC_MOVE_SIGMA_BIRTH;
    int &n = sig ? k : l;
    const LdsColumn z{sig ? zc.p : zm.p, T}, v{sig ? ph.p : mm.p, T};
    if (n < (sig ? kc : km)) {
      const double zn = sh.z_max * u1;
      const double vn = sig ? affine(pr.phi_lo, pr.phi_hi, u2) : affine(pr.m_lo, pr.m_hi, u2);
      int j = 0;
      while (j < n && z[j] < zn) ++j;
      for (int q = n; q > j; --q) {
        z[q] = z[q - 1];
        v[q] = v[q - 1];
      }
      z[j] = zn;
      v[j] = vn;
      ++n;
      ok = true;
    }
  } else if (t == RJSMC_MOVE_SIGMA_DEATH || t == RJSMC_MOVE_M_DEATH) {
    const bool sig = t == RJSMC_MOVE_SIGMA_DEATH;
    int &n = sig ? k : l;
    const LdsColumn z{sig ? zc.p : zm.p, T}, v{sig ? ph.p : mm.p, T};
    if (n > 0) {
      int j = (int)(u1 * (double)n);
      j = j > n - 1 ? n - 1 : j;
      for (int q = j; q + 1 < n; ++q) {
        z[q] = z[q + 1];
        v[q] = v[q + 1];
      }
      --n;
      ok = true;
    }
  } else if (t == RJSMC_MOVE_SIGMA_MOVE || t == RJSMC_MOVE_M_MOVE) {
    const bool sig = t == RJSMC_MOVE_SIGMA_MOVE;
    const int n = sig ? k : l;
    const LdsColumn z{sig ? zc.p : zm.p, T};
    if (n > 0) {
      int j = (int)(u1 * (double)n);
      j = j > n - 1 ? n - 1 : j;
      const double zn = madd_rn(z[j], a.z_move_sd, nz);
      const double lo = j > 0 ? z[j - 1] : 0.0;
      const double hi = j + 1 < n ? z[j + 1] : sh.z_max;
      if (lo < zn && zn < hi && zn > 0.0) {
        z[j] = zn;
        ok = true;
      }
    }
  } else if (t == RJSMC_MOVE_WITHIN_RW) {
    const double step = rw_scale * nz;
    // theta' = theta + step F[:, r] in parameter-vector order (phi_b, phi, z_cond, m,
    // z_charg, log10 tau, c); the layer entries are loaded together, not one per update
    madd_rows2(ph, zc, Fr + 1, Fr + 1 + k, k, step);
    madd_rows2(mm, zm, Fr + 1 + 2 * k, Fr + 1 + 2 * k + l, l, step);
    phb = madd_rn(phb, step, f0);
    lt = madd_rn(lt, step, fa);
    cc = madd_rn(cc, step, fb);
    ok = in_range(phb, pr.phi_lo, pr.phi_hi) && in_range(lt, pr.ltau_lo, pr.ltau_hi) &&
         in_range(cc, pr.c_lo, pr.c_hi);
    for (int j = 0; j < k; ++j)
      ok = ok && in_range(ph[j], pr.phi_lo, pr.phi_hi) && zc[j] > 0.0 && zc[j] < sh.z_max &&
           (j == 0 || zc[j] > zc[j - 1]);
    for (int j = 0; j < l; ++j)
      ok = ok && in_range(mm[j], pr.m_lo, pr.m_hi) && zm[j] > 0.0 && zm[j] < sh.z_max &&
           (j == 0 || zm[j] > zm[j - 1]);
  } else if (MALA && t == RJSMC_MOVE_WITHIN_MALA) {
    const int d = 3 + 2 * k + 2 * l, D = sh.dmax;
    const int mdl = k * (km + 1) + l;
    const double *Fm = a.factors + (snd * sh.n_models + mdl) * (int64_t)D * D;   // F[a][r] = Fm[r D + a]
    const double gam = gamma[snd];
    double th[kDimMax], xi[kDimMax], cr[kDimMax];
    for (int q = 0; q < d; ++q) th[q] = theta_get(st, i, k, l, q);
    mala_normals(a, i, move, d, xi);
    const double eps = a.mala_eps_dev ? a.mala_eps_dev[snd] : a.mala_eps;
    for (int r = 0; r < d; ++r) {          // cr = eps^2/2 F^T (gamma grad) + eps xi
      double sr = 0.0;
      for (int q = 0; q < d; ++q) sr += Fm[r * D + q] * (gam * theta_get(gcur, i, k, l, q));
      cr[r] = 0.5 * eps * eps * sr + eps * xi[r];
    }
    for (int q = 0; q < d; ++q) {
      double acc = 0.0;
      for (int r = 0; r < d; ++r) acc += Fm[r * D + q] * cr[r];
      th[q] += acc;
    }
    int q = 0;
    phb = th[q++];
    for (int j = 0; j < k; ++j) ph[j] = th[q++];
    for (int j = 0; j < k; ++j) zc[j] = th[q++];
    for (int j = 0; j < l; ++j) mm[j] = th[q++];
    for (int j = 0; j < l; ++j) zm[j] = th[q++];
    lt = th[q++];
    cc = th[q++];
    ok = in_range(phb, pr.phi_lo, pr.phi_hi) && in_range(lt, pr.ltau_lo, pr.ltau_hi) &&
         in_range(cc, pr.c_lo, pr.c_hi);
    for (int j = 0; j < k; ++j)
      ok = ok && in_range(ph[j], pr.phi_lo, pr.phi_hi) && zc[j] > 0.0 && zc[j] < sh.z_max &&
           (j == 0 || zc[j] > zc[j - 1]);
    for (int j = 0; j < l; ++j)
      ok = ok && in_range(mm[j], pr.m_lo, pr.m_hi) && zm[j] > 0.0 && zm[j] < sh.z_max &&
           (j == 0 || zm[j] > zm[j - 1]);
  }
  mask[i] = ok ? (t == RJSMC_MOVE_WITHIN_MALA ? 2 : 1) : 0;
  if (!ok) return;
  prop.kappa[i] = k;
  prop.lambda[i] = l;
  prop.phi_b[i] = phb;
  prop.log10_tau[i] = lt;
  prop.c[i] = cc;
  for (int j = 0; j < kc; ++j) {
    prop.z_cond[j * So + i] = j < k ? zc[j] : 0.0;
    prop.phi[j * So + i] = j < k ? ph[j] : 0.0;
  }
  for (int j = 0; j < km; ++j) {
    prop.z_charg[j * So + i] = j < l ? zm[j] : 0.0;
    prop.m[j * So + i] = j < l ? mm[j] : 0.0;
  }
}

template <bool MALA, bool ZCA>
__global__ __launch_bounds__(256) void propose_kernel(SmcShape sh, rjsmc_mutate_args a, int move, DevParticles st,
                                                      DevParticlesW prop, int32_t *mask, int32_t *type,
                                                      const double *gamma, DevParticles gcur, int32_t *gvalid,
                                                      double *lq, const int32_t *active, int draw) {
  propose_particle<MALA, ZCA>((int64_t)blockIdx.x * blockDim.x + threadIdx.x, sh, a, move, st, prop, mask, type, gamma,
                              gcur, gvalid, lq, active, draw);
}

// Metropolis-Hastings decision: accept when ln u < gamma (ll' - ll).  Every thread of a
// wave takes part (the tallies are wave ballots).
__device__ __forceinline__ void accept_particle(int64_t i, const SmcShape &sh, const rjsmc_mutate_args &a, int move,
                                                const DevParticlesW &st, double *ll, const DevParticles &prop,
                                                const double *ll_prop, const int32_t *mask, const int32_t *type,
                                                const double *gamma, const DevParticlesW &gcur,
                                                const DevParticles &gprop, int32_t *gvalid, int64_t *stats,
                                                const double *lq) {
  const bool in = i < st.n;
  const int t = in ? type[i] : -1;
  bool acc = false;
  if (in && t >= 0 && mask[i]) {
    const int64_t snd = st.n_per_sounding > 0 ? i / st.n_per_sounding : 0;
    double u0, ua;
    uniforms(a.seed, (uint32_t)i, (uint32_t)step_of(a), (uint32_t)move, 0u, u0, ua);
    double extra = 0.0;
    if (t == RJSMC_MOVE_WITHIN_MALA) {
      // log q(theta | theta') - log q(theta' | theta) = -|xi + eps/2 F^T gamma (g + g')|^2/2 + |xi|^2/2
      const int k = st.kappa[i], l = st.lambda[i];
      const int d = 3 + 2 * k + 2 * l, D = sh.dmax;
      const double *Fm = a.factors + (snd * sh.n_models + (k * (sh.km + 1) + l)) * (int64_t)D * D;
      const double gam = gamma[snd];
      const double eps = a.mala_eps_dev ? a.mala_eps_dev[snd] : a.mala_eps;
      double xi[kDimMax];
      mala_normals(a, i, move, d, xi);
      for (int r = 0; r < d; ++r) {
        double sr = 0.0;
        for (int q = 0; q < d; ++q)
          sr += Fm[r * D + q] * (gam * (theta_get(readonly(gcur), i, k, l, q) + theta_get(gprop, i, k, l, q)));
        const double v = xi[r] + 0.5 * eps * sr;
        extra += -0.5 * v * v + 0.5 * xi[r] * xi[r];
      }
    }
    if (a.zca_birth && lq &&
        (t == RJSMC_MOVE_SIGMA_BIRTH || t == RJSMC_MOVE_M_BIRTH || t == RJSMC_MOVE_SIGMA_DEATH ||
         t == RJSMC_MOVE_M_DEATH))
      extra += lq[i];                     // adaptive birth / death: proposal and Jacobian terms
    const double margin = gamma[snd] * (ll_prop[i] - ll[i]) + extra - log(ua);
    acc = margin > 0.0;
    if (acc && a.trial == 0) {
      const int64_t S = st.stride, Sp = prop.stride;
      const int pk = prop.kappa[i], pl = prop.lambda[i];
      const double pb = prop.phi_b[i], pt = prop.log10_tau[i], pc = prop.c[i];
      st.kappa[i] = pk;
      st.lambda[i] = pl;
      st.phi_b[i] = pb;
      st.log10_tau[i] = pt;
      st.c[i] = pc;
      copy_rows2(st.z_cond, st.phi, S, prop.z_cond, prop.phi, Sp, i, sh.kc);
      copy_rows2(st.z_charg, st.m, S, prop.z_charg, prop.m, Sp, i, sh.km);
      ll[i] = ll_prop[i];
      if (gvalid) {
        // a Langevin proposal brings its own gradient; any other accepted move leaves the
        // cached gradient stale
        if (t == RJSMC_MOVE_WITHIN_MALA) {
          const int64_t Sg = gcur.stride, Sq = gprop.stride;
          gcur.phi_b[i] = gprop.phi_b[i];
          gcur.log10_tau[i] = gprop.log10_tau[i];
          gcur.c[i] = gprop.c[i];
          for (int j = 0; j < sh.kc; ++j) {
            gcur.phi[j * Sg + i] = gprop.phi[j * Sq + i];
            gcur.z_cond[j * Sg + i] = gprop.z_cond[j * Sq + i];
          }
          for (int j = 0; j < sh.km; ++j) {
            gcur.m[j * Sg + i] = gprop.m[j * Sq + i];
            gcur.z_charg[j * Sg + i] = gprop.z_charg[j * Sq + i];
          }
        } else {
          gvalid[i] = 0;
        }
      }
    }
  }
  if (a.stats_sound && (t == RJSMC_MOVE_WITHIN_RW || t == RJSMC_MOVE_WITHIN_MALA)) {
    // every drawn within-model proposal counts, also one that leaves the support
    const int64_t snd = st.n_per_sounding > 0 ? i / st.n_per_sounding : 0;
    atomicAdd((unsigned long long *)&a.stats_sound[2 * snd], 1ull);
    if (acc) atomicAdd((unsigned long long *)&a.stats_sound[2 * snd + 1], 1ull);
  }
  if (stats) {
    const int lane = threadIdx.x & (kWave - 1);
    for (int q = 0; q < RJSMC_N_MOVES; ++q) {
      const int np = __popcll(__ballot(t == q));
      const int na = __popcll(__ballot(t == q && acc));
      if (lane == 0 && np) atomicAdd((unsigned long long *)&stats[q], (unsigned long long)np);
      if (lane == 0 && na) atomicAdd((unsigned long long *)&stats[RJSMC_N_MOVES + q], (unsigned long long)na);
    }
  }
}

__global__ __launch_bounds__(256) void accept_kernel(SmcShape sh, rjsmc_mutate_args a, int move, DevParticlesW st,
                                                     double *ll, DevParticles prop, const double *ll_prop,
                                                     const int32_t *mask, const int32_t *type, const double *gamma,
                                                     DevParticlesW gcur, DevParticles gprop, int32_t *gvalid,
                                                     int64_t *stats, const double *lq) {
  accept_particle((int64_t)blockIdx.x * blockDim.x + threadIdx.x, sh, a, move, st, ll, prop, ll_prop, mask, type, gamma,
                  gcur, gprop, gvalid, stats, lq);
}

// The decision of sweep move_prev, then the proposal of sweep move, for every particle:
// both read and write only the particle's own state, proposal, move type, mask and
// correction (each read before it is rewritten), so one launch serves the two.  Sweeps
// without gradient-informed moves only.  The decision is accept_particle's; the launch
// loads everything either step reads in one round, before the decision: the current
// state (scalars in registers, layer rows, all rows up to the capacities, into the
// proposal's LDS columns), the decision's inputs, and, for an evaluated proposal, the
// proposal itself, so that an accepted one is copied from registers and the next
// proposal starts from whichever state survives without reading it back.
template <bool ZCA>
__global__ __launch_bounds__(256) void accept_propose_kernel(SmcShape sh, rjsmc_mutate_args a, int move_prev, int move,
                                                             DevParticlesW st_w, DevParticles st_r, double *ll,
                                                             DevParticles prop_r, DevParticlesW prop_w,
                                                             const double *ll_prop, int32_t *mask, int32_t *type,
                                                             const double *gamma, int64_t *stats, double *lq,
                                                             const int32_t *active) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i < st_r.n;
  const int kc = sh.kc, km = sh.km;
  const int64_t S = st_r.stride, Sp = prop_r.stride;
  const int64_t snd = in && st_r.n_per_sounding > 0 ? i / st_r.n_per_sounding : 0;
  extern __shared__ double prop_lds[];
  const int T = blockDim.x;
  double *lds0 = prop_lds + threadIdx.x;
  const LdsColumn zc{lds0, T}, ph{lds0 + (int64_t)kc * T, T}, zm{lds0 + (int64_t)2 * kc * T, T},
      mm{lds0 + (int64_t)(2 * kc + km) * T, T};
  StateRegs s0{0, 0, 0.0, 0.0, 0.0};
  int t = -1, mk = 0;
  double llp = 0.0, llc = 0.0, gm = 0.0, lqv = 0.0;
  if (in) {
    t = type[i];
    mk = mask[i];
    llp = ll_prop[i];
    llc = ll[i];
    gm = gamma[snd];
    if (ZCA && lq) lqv = lq[i];
    s0.k = st_r.kappa[i];
    s0.l = st_r.lambda[i];
    s0.phb = st_r.phi_b[i];
    s0.lt = st_r.log10_tau[i];
    s0.cc = st_r.c[i];
    load_rows2(st_r.z_cond, st_r.phi, S, i, kc, zc, ph);
    load_rows2(st_r.z_charg, st_r.m, S, i, km, zm, mm);
  }
  bool acc = false;
  if (in && t >= 0 && mk) {
    const bool copy = a.trial == 0;
    // the proposal (the next state if accepted), the first kRowBatch rows in registers
    int pk = 0, pl = 0;
    double pb = 0.0, pt = 0.0, pc = 0.0;
    double rz[kRowBatch], rp[kRowBatch], rzm[kRowBatch], rmm[kRowBatch];
    if (copy) {
      pk = prop_r.kappa[i];
      pl = prop_r.lambda[i];
      pb = prop_r.phi_b[i];
      pt = prop_r.log10_tau[i];
      pc = prop_r.c[i];
#pragma unroll
      for (int j = 0; j < kRowBatch; ++j) {
        rz[j] = j < kc ? prop_r.z_cond[(int64_t)j * Sp + i] : 0.0;
        rp[j] = j < kc ? prop_r.phi[(int64_t)j * Sp + i] : 0.0;
        rzm[j] = j < km ? prop_r.z_charg[(int64_t)j * Sp + i] : 0.0;
        rmm[j] = j < km ? prop_r.m[(int64_t)j * Sp + i] : 0.0;
      }
    }
    double u0, ua;
    uniforms(a.seed, (uint32_t)i, (uint32_t)step_of(a), (uint32_t)move_prev, 0u, u0, ua);
    double extra = 0.0;
    if (ZCA && a.zca_birth && lq &&
        (t == RJSMC_MOVE_SIGMA_BIRTH || t == RJSMC_MOVE_M_BIRTH || t == RJSMC_MOVE_SIGMA_DEATH ||
         t == RJSMC_MOVE_M_DEATH))
      extra += lqv;                       // adaptive birth / death: proposal and Jacobian terms
    const double margin = gm * (llp - llc) + extra - log(ua);
    acc = margin > 0.0;
    if (acc && copy) {
      st_w.kappa[i] = pk;
      st_w.lambda[i] = pl;
      st_w.phi_b[i] = pb;
      st_w.log10_tau[i] = pt;
      st_w.c[i] = pc;
#pragma unroll
      for (int j = 0; j < kRowBatch; ++j) {
        if (j < kc) {
          st_w.z_cond[(int64_t)j * S + i] = rz[j];
          st_w.phi[(int64_t)j * S + i] = rp[j];
          zc[j] = rz[j];
          ph[j] = rp[j];
        }
        if (j < km) {
          st_w.z_charg[(int64_t)j * S + i] = rzm[j];
          st_w.m[(int64_t)j * S + i] = rmm[j];
          zm[j] = rzm[j];
          mm[j] = rmm[j];
        }
      }
      // rows beyond the first batch (capacities above kRowBatch)
      for (int j = kRowBatch; j < kc; ++j) {
        const double z = prop_r.z_cond[(int64_t)j * Sp + i], v = prop_r.phi[(int64_t)j * Sp + i];
        st_w.z_cond[(int64_t)j * S + i] = z;
        st_w.phi[(int64_t)j * S + i] = v;
        zc[j] = z;
        ph[j] = v;
      }
      for (int j = kRowBatch; j < km; ++j) {
        const double z = prop_r.z_charg[(int64_t)j * Sp + i], v = prop_r.m[(int64_t)j * Sp + i];
        st_w.z_charg[(int64_t)j * S + i] = z;
        st_w.m[(int64_t)j * S + i] = v;
        zm[j] = z;
        mm[j] = v;
      }
      ll[i] = llp;
      s0 = StateRegs{pk, pl, pb, pt, pc};
    }
  }
  if (a.stats_sound && (t == RJSMC_MOVE_WITHIN_RW || t == RJSMC_MOVE_WITHIN_MALA)) {
    // every drawn within-model proposal counts, also one that leaves the support
    atomicAdd((unsigned long long *)&a.stats_sound[2 * snd], 1ull);
    if (acc) atomicAdd((unsigned long long *)&a.stats_sound[2 * snd + 1], 1ull);
  }
  if (stats) {
    const int lane = threadIdx.x & (kWave - 1);
    for (int q = 0; q < RJSMC_N_MOVES; ++q) {
      const int np = __popcll(__ballot(t == q));
      const int na = __popcll(__ballot(t == q && acc));
      if (lane == 0 && np) atomicAdd((unsigned long long *)&stats[q], (unsigned long long)np);
      if (lane == 0 && na) atomicAdd((unsigned long long *)&stats[RJSMC_N_MOVES + q], (unsigned long long)na);
    }
  }
  propose_particle<false, ZCA>(i, sh, a, move, st_r, prop_w, mask, type, gamma, DevParticles(), nullptr, lq, active, 1,
                               &s0);
}

hipError_t launch_draw_types(const rjsmc_mutate_args &a, int move, const DevParticles &state, int kc, int km,
                             int32_t *mask, int32_t *type, const int32_t *active, const int32_t *gvalid,
                             hipStream_t stream) {
  const int64_t blocks = (state.n + 255) / 256;
  hipLaunchKernelGGL(draw_types_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, a, move, state, kc, km, mask,
                     type, active, gvalid);
  return hipGetLastError();
}

__global__ void fill_i32_kernel(int32_t *p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t stream) {
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, n, v);
  return hipGetLastError();
}

hipError_t launch_propose(const SmcShape &sh, const rjsmc_mutate_args &a, int move, const DevParticles &state,
                          const DevParticlesW &prop, int32_t *mask, int32_t *type, const double *gamma,
                          const DevParticles *grad_cur, int32_t *gvalid, double *lq, const int32_t *active,
                          bool draw, hipStream_t stream) {
  // the four layer arrays of each thread in LDS; 256 threads per workgroup (as the kernels
  // before and after it, so that a small population stays on one compute unit and its L2)
  // unless the arrays of the largest capacities need fewer
  const size_t per_thread = sizeof(double) * (size_t)(2 * sh.kc + 2 * sh.km);
  const int kThreads = per_thread * 256 <= 64 * 1024 ? 256 : kWave;
  const int64_t blocks = (state.n + kThreads - 1) / kThreads;
  const size_t lds = per_thread * kThreads;
  const DevParticles g = grad_cur ? *grad_cur : DevParticles();
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(kThreads), lds, stream, sh, a, move, state, prop, mask,
                       type, gamma, g, gvalid, lq, active, draw ? 1 : 0);
  };
  const bool mala = grad_cur != nullptr, zca = a.zca_birth != 0;
  if (mala && zca)
    go(propose_kernel<true, true>);
  else if (mala)
    go(propose_kernel<true, false>);
  else if (zca)
    go(propose_kernel<false, true>);
  else
    go(propose_kernel<false, false>);
  return hipGetLastError();
}

hipError_t launch_accept_propose(const SmcShape &sh, const rjsmc_mutate_args &a, int move_prev, int move,
                                 const DevParticlesW &state, double *ll, const DevParticlesW &prop,
                                 const double *ll_prop, int32_t *mask, int32_t *type, const double *gamma,
                                 int64_t *stats, double *lq, const int32_t *active, hipStream_t stream) {
  // the proposal's launch shape and LDS (launch_propose)
  const size_t per_thread = sizeof(double) * (size_t)(2 * sh.kc + 2 * sh.km);
  const int kThreads = per_thread * 256 <= 64 * 1024 ? 256 : kWave;
  const int64_t blocks = (state.n + kThreads - 1) / kThreads;
  const size_t lds = per_thread * kThreads;
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(kThreads), lds, stream, sh, a, move_prev, move, state,
                       readonly(state), ll, readonly(prop), prop, ll_prop, mask, type, gamma, stats, lq, active);
  };
  if (a.zca_birth)
    go(accept_propose_kernel<true>);
  else
    go(accept_propose_kernel<false>);
  return hipGetLastError();
}

hipError_t launch_accept(const SmcShape &sh, const rjsmc_mutate_args &a, int move, const DevParticlesW &state,
                         double *ll, const DevParticles &prop, const double *ll_prop, const int32_t *mask,
                         const int32_t *type, const double *gamma, const DevParticlesW *grad_cur,
                         const DevParticles *grad_prop, int32_t *gvalid, int64_t *stats, const double *lq,
                         hipStream_t stream) {
  const int64_t blocks = (state.n + 255) / 256;
  const DevParticlesW gc = grad_cur ? *grad_cur : DevParticlesW();
  const DevParticles gp = grad_prop ? *grad_prop : DevParticles();
  hipLaunchKernelGGL(accept_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, sh, a, move, state, ll, prop,
                     ll_prop, mask, type, gamma, gc, gp, grad_cur ? gvalid : nullptr, stats, lq);
  return hipGetLastError();
}

// -------------------------------------------------------------- posterior summaries ---
// Grid (sounding, item block): item j < M counts the particles of model j; item M the
// chargeable-versus-conductive Bayes factor; items M + 1 + d the depth profiles at
// depth d.  Each item walks the sounding's particles in index order (deterministic sums).
__global__ __launch_bounds__(256) void summary_kernel(SmcShape sh, DevParticles p, rjsmc_summary_args a) {
  const int s = blockIdx.x;
  const int j = blockIdx.y * blockDim.x + threadIdx.x;
  const int M = sh.n_models;
  if (j >= M + 1 + a.n_depth) return;
  const int64_t N = p.n_per_sounding > 0 ? p.n_per_sounding : p.n;
  const int64_t off = (int64_t)s * N, S = p.stride;
  const bool dec = p.layout == RJSMC_LAYOUT_DECOUPLED;
  if (j < M) {
    if (!a.model_count) return;
    int cnt = 0;
    for (int64_t q = 0; q < N; ++q) {
      const int64_t i = off + q;
      const int lam = dec ? p.lambda[i] : 0;
      cnt += p.kappa[i] * (sh.km + 1) + lam == j;
    }
    a.model_count[(int64_t)s * M + j] = cnt;
    return;
  }
  if (j == M) {
    if (!a.log_bfipd) return;
    if (!dec || sh.km == 0) {
      a.log_bfipd[s] = __builtin_nan("");
      return;
    }
    int64_t non = 0;
    for (int64_t q = 0; q < N; ++q) non += p.lambda[off + q] == 0;
    // (mean posterior-to-prior ratio over chargeable models) / (the same over conductive
    // models), uniform model prior: (n_charg / n_cond) |M_cond| / |M_charg|, with
    // |M_cond| = kmax_cond + 1 and |M_charg| = (kmax_cond + 1) kmax_charg
    a.log_bfipd[s] = log((double)(N - non)) - log((double)non) - log((double)sh.km);
    return;
  }
  const int d = j - M - 1;
  const double z = a.depth_m[d];
  double sphi = 0.0, sm = 0.0;
  int64_t npos = 0;
  for (int64_t q = 0; q < N; ++q) {
    const int64_t i = off + q;
    const int kap = p.kappa[i];
    int ic = 0;
    for (int r = 0; r < kap; ++r) ic += p.z_cond[r * S + i] <= z;
    const double phi = ic == 0 ? p.phi_b[i] : p.phi[(int64_t)(ic - 1) * S + i];
    double m;
    if (dec) {
      const int lam = p.lambda[i];
      int im = 0;
      for (int r = 0; r < lam; ++r) im += p.z_charg[r * S + i] <= z;
      m = im == 0 ? 0.0 : p.m[(int64_t)(im - 1) * S + i];
    } else {
      m = p.m[(int64_t)ic * S + i];
    }
    sphi += phi;
    sm += m;
    npos += m > 0.0;
  }
  const int64_t o = (int64_t)s * a.n_depth + d;
  if (a.mean_log10_sigma) a.mean_log10_sigma[o] = sphi / (double)N;
  if (a.mean_m) a.mean_m[o] = sm / (double)N;
  if (a.p_chargeable) a.p_chargeable[o] = (double)npos / (double)N;
}

hipError_t launch_summary(const SmcShape &sh, const DevParticles &p, const rjsmc_summary_args &a, hipStream_t stream) {
  const int items = sh.n_models + 1 + a.n_depth;
  hipLaunchKernelGGL(summary_kernel, dim3((unsigned)a.n_sound, (unsigned)((items + 255) / 256)), dim3(256), 0, stream,
                     sh, p, a);
  return hipGetLastError();
}

// ------------------------------------------------- posterior predictive summaries ---
// One thread per (sounding, gate); the sounding's particles are summed in index order
// (two passes: the mean, then the spread about it and the noise variances).
__global__ __launch_bounds__(256) void ppd_kernel(int64_t N, int n_sound, int ng, const double *resp,
                                                  const double *eps_an2, double eps_mn, const double *y_obs,
                                                  double *mean, double *sd, double *z) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n_sound * ng) return;
  const int64_t s = t / ng;
  const int g = (int)(t - s * ng);
  const double *y = resp + s * N * ng + g;
  double sum = 0.0;
  for (int64_t i = 0; i < N; ++i) sum += y[i * ng];
  const double mu = sum / (double)N;
  double spread = 0.0, noise = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    const double yi = y[i * ng], dy = yi - mu, e = eps_mn * yi;
    spread += dy * dy;
    noise += eps_an2[g] + e * e;
  }
  const double sdv = sqrt(spread / (double)N + noise / (double)N);
  mean[t] = mu;
  sd[t] = sdv;
  if (z) z[t] = (y_obs[t] - mu) / sdv;
}

hipError_t launch_ppd(const DevSystem &sys, const DevParticles &p, int n_sound, const double *resp,
                      const double *y_obs, double *mean, double *sd, double *z, hipStream_t stream) {
  const int64_t N = p.n_per_sounding > 0 ? p.n_per_sounding : p.n;
  const int64_t items = (int64_t)n_sound * sys.n_gate;
  hipLaunchKernelGGL(ppd_kernel, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, stream, N, n_sound, sys.n_gate,
                     resp, sys.eps_an2, sys.eps_mn, y_obs, mean, sd, z);
  return hipGetLastError();
}

// ------------------------------------------------------------ step-size bisection ---
__global__ void scale_bisect_kernel(rjsmc_bisect_args a) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.n_sound) return;
  double lo, hi;
  if (a.init) {
    lo = log(a.lo0);
    hi = log(a.hi0);
  } else {
    lo = a.log_lo[s];
    hi = a.log_hi[s];
    const int64_t tried = a.stats_sound[2 * s], taken = a.stats_sound[2 * s + 1];
    if (tried > 0) {
      const double mid = 0.5 * (lo + hi);
      if ((double)taken / (double)tried > a.target)
        lo = mid;
      else
        hi = mid;
    }
  }
  a.log_lo[s] = lo;
  a.log_hi[s] = hi;
  a.scale[s] = exp(0.5 * (lo + hi));
  a.stats_sound[2 * s] = 0;
  a.stats_sound[2 * s + 1] = 0;
}

hipError_t launch_scale_bisect(const rjsmc_bisect_args &a, hipStream_t stream) {
  hipLaunchKernelGGL(scale_bisect_kernel, dim3((unsigned)((a.n_sound + 255) / 256)), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace rjsmc
