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
  for (int t = threadIdx.x; t < nf; t += blockDim.x) s_omega[t] = s.omega[t];
  for (int t = threadIdx.x; t < nf * ng; t += blockDim.x) s_K[t] = s.K[t];
  for (int t = threadIdx.x; t < ng; t += blockDim.x) s_eps2[t] = s.eps_an2[t];
  for (int t = threadIdx.x; t < kPhaseN; t += blockDim.x)
    s_phase[t] = cplx<double>{s.phase[2 * t], s.phase[2 * t + 1]};
  for (int t = threadIdx.x; t < kExp2N; t += blockDim.x) s_exp2[t] = s.exp2t[t];
  LayerStack *st = &s_stack[wave];
  __syncthreads();
  const int L = merge_particle(p, i, valid && !skip, kc, km, LMAX, st, s.flags);

  // per-particle Cole-Cole constants: (i w tau)^c = (w tau)^c (cos(pi c/2) + i sin(pi c/2))
  double c = 0.0, log_tau = 0.0, spc = 0.0, cpc = 1.0;
  if (L > 0) {
    c = p.c[i];
    log_tau = p.log10_tau[i] * 2.302585092994045684;
    sincospi(0.5 * c, &spc, &cpc);
    if (lane < L - 1) s_h2[wave][lane] = T(-2) * to<T>(st->top[lane + 1] - st->top[lane]);
  }
  const int gl = lane & 7, gw = lane >> 3;
  const int nhg = nhp >> 3;
  const int nq = (nf + 7) >> 3;
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
    if (act) {
      const double w = s_omega[jf];
      // q_cc = 1 / (1 + (i w tau)^c); k2 = i w mu0 sigma_inf (1 - m q_cc)
      const double pw = exp(c * (log(w) + log_tau));
      const cplx<double> qcc = crcp(cplx<double>{1.0 + pw * cpc, pw * spc});
      const T wmu = to<T>(w * kMu0);
      const cplx<T> qt = {to<T>(qcc.re), to<T>(qcc.im)};
      auto k2_of = [&](int l) {
        const T sg = to<T>(st->sig[l]), mg = to<T>(st->m[l]);
        const cplx<T> sh = {sg * (T(1) - mg * qt.re), sg * (-(mg * qt.im))};
        return cplx<T>{-(wmu * sh.im), wmu * sh.re};
      };
      for (int l = gl; l < L; l += 8) {
        const cplx<T> kl = k2_of(l);
        s_k2[wave][gw][l] = kl;
        if (l + 1 < L) s_dk2[wave][gw][l] = kl - k2_of(l + 1);
      }
    }
    wave_lds_sync();
    if (act && A == 1) {
      double acc = 0.0;
#pragma unroll 1
      for (int sidx = 0; sidx < nhg; ++sidx) {
        const int k = gl + 8 * sidx;
        const T rim = reflection_im<T>(to<T>(s_lam[k]), s_k2[wave][gw], s_dk2[wave][gw], s_h2[wave], L,
                                         s_phase, s_exp2);
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
                                                                   s_exp2));
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
  if (L > 0) {
    double term = 0.0;
    if (lane < ng) {
      double y = 0.0;
      for (int j = 0; j < nf; ++j) y += s_K[lane * nf + j] * s_imh[pw][j];
      if (resp) resp[i * ng + lane] = y;
      if (ll) {
        const int64_t snd = p.n_per_sounding > 0 ? i / p.n_per_sounding : 0;
        const double d = y_obs[snd * ng + lane];
        const double e = s.eps_mn * y;
        const double s2 = s_eps2[lane] + e * e;
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
  } else if (valid && !skip) {
    // invalid particle: NaN responses, -inf log-likelihood
    if (resp && lane < ng) resp[i * ng + lane] = __builtin_nan("");
    if (ll && lane == 0) ll[i] = -HUGE_VAL;
  }
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
  RJSMC_TILE_DISPATCH(launch_t, T, t.waves_per_block, t.waves_per_particle, s, p, kc, km, resp, y_obs, ll, t.perm,
                      stream);
}

template <typename T>
static hipError_t lds_prec(const DevSystem &s, int w, int q, size_t *bytes) {
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
