// Log-likelihood and its gradient (reverse sweep) for gfx950.
//
// One wavefront per particle, lanes tiling (frequency, filter abscissa) as in the
// forward kernel, and every (frequency, abscissa) pair visited once.  Per pair the lane
// runs the projective reflection recursion bottom-up, keeping the state (N_l, D_l) of
// every interface (of every even one at 12 and 16 layers, the odd ones rebuilt on the
// way back) in a per-lane array held in registers (the layer loops unrolled over the
// instantiation's capacity: 4, 8, 12 or 16 merged layers; at 12 and 16 a few values
// spill at two waves per SIMD); the same recursion gives Im r_TE for the Hankel sum.
// It then sweeps top-down through the surface and every interface, propagating the
// adjoint of c_k Im r (the reverse sweep is linear in its seed, so the filter coefficient
// alone seeds it) and accumulating, per lane and frequency, the complex adjoints of the
// layer wavenumbers k2_l = i w mu0 sigma_hat_l and the adjoints of the thicknesses.  The
// u_l and E_l of the recursion are recomputed in the sweep instead of stored.  Per
// frequency these derivatives of Im H(w_j) are mapped through the Cole-Cole terms to a
// slot vector u_j over (log10 sigma_inf, m) of each merged layer, the thicknesses and
// (log10 tau, c), kept in LDS (as they are, or folded into the gates' sums
// V_g = sum_j K_gj u_j); once the gates and the likelihood are formed, the gradient is
// sum_j wbar_j u_j = sum_g ybar_g V_g with ybar_g = d ll / d y_g and
// wbar_j = sum_g K_gj ybar_g, and the merged-layer gradients are routed back to the
// particle's parameters through the merge (an interface moves the thickness above and
// below it).
#include <hip/hip_runtime.h>

#include "cplx.h"
#include "merge.h"
#include "recursion.h"
#include "rjsmc_internal.h"

namespace rjsmc {

namespace {
constexpr int kWavesA = 2;                               // particles per block
constexpr int64_t kBucketMin = 4096;   // fewer particles: one launch (the sort costs more than it saves)
constexpr double kMu0A = 1.25663706143591729539e-06;
constexpr double kTwoPiA = 6.28318530717958647692;
constexpr double kLn10 = 2.302585092994045684;
constexpr double kHalfPi = 1.57079632679489661923;
}  // namespace

__device__ __forceinline__ cplx<double> crcp_fast(cplx<double> b) {
  const double inv = fast_rcp(b.re * b.re + b.im * b.im);
  return {b.re * inv, -b.im * inv};
}
__device__ __forceinline__ cplx<double> cdiv_fast(cplx<double> a, cplx<double> b) { return a * crcp_fast(b); }

// u = sqrt(z), the principal root as csqrt_fast forms it, and hm = 1/(2|z|), so that
// 1/(2u) = conj(u) hm (|u|^2 = |z|): the refined reciprocal square root of |z|^2 that
// gives |z| gives hm as well.
__device__ __forceinline__ cplx<double> csqrt_hm(cplx<double> z, double &hm) {
  double mag;
  sqrt_hrsqrt(z.re * z.re + z.im * z.im, mag, hm);
  const double w = 0.5 * (mag + fabs(z.re));
  double t, ht;
  sqrt_hrsqrt(w, t, ht);
  const double o = z.im * ht;   // Im z / (2 t)
  const bool right = z.re >= 0.0;
  return {right ? t : fabs(o), right ? o : copysign(t, z.im)};
}

// Adds the adjoints of one (lam, w) pair with seed wt (the weight of Im r) to
// G[l] (d(wt r)/d k2_l) and H[l] (Im d(wt r)/d h_l).  The bottom-up pass is the forward's
// projective recursion (step_up), keeping the state (N_l, D_l) of the interfaces; the
// top-down pass applies the adjoint of each step: for N' = a S - b T, D' = a S + b T,
// S = D + N E, T = D - N E and output adjoints N'~, D'~,
//   P~ = N'~ + D'~,  Q~ = D'~ - N'~,  a~ += P~ S,  b~ += Q~ T,
//   S~ = P~ a,  T~ = Q~ b,  D~ = S~ + T~,  N~ = (S~ - T~) E,  E~ = (S~ - T~) N,
// with E = exp(h2 u) (h2 = -2 h): u~ += E~ h2 E and h~ = -2 u E~ E.  The seed is
// N~ = wt / D, D~ = -N~ N / D at the surface, and u_l = sqrt(lam^2 + k2_l) gives
// k2_l~ += u_l~ / (2 u_l).  The 12- and 16-layer instantiations keep the states of the
// even interfaces only and rebuild an odd one, when the top-down pass reaches it, by one
// step up from the state below it (the u and E of that step are the next step's, so
// they are formed once): half the registers for the states, for one step up per two
// layers.  One complex reciprocal per pair, and 1/(2 u_l) per layer:
// the 12- and 16-layer instantiations take it from the square root's own 1/(2|u_l|^2)
// (two products; 3% faster there), the smaller ones form a complex reciprocal at the
// point of use (one register pair fewer through the sweep keeps them within 256 VGPRs
// unspilled).  u_l and E_l are recomputed in the top-down pass instead of stored.
template <int LMAX>
__device__ __forceinline__ void pair_adjoint(double lam, const cplx<double> *k2, const double *h2v, int L,
                                             double wt, cplx<double> (&G)[LMAX], double (&H)[LMAX],
                                             const cplx<double> *phase, const double *e2, double &imr) {
  const double lam2 = lam * lam;
  // The layer loops are unrolled over LMAX with a wave-uniform guard, so the stored
  // states, G and H stay in registers (at 12 and 16 layers some of them spill at two
  // waves per SIMD: still faster than indexing them in private memory).
  constexpr int NI = LMAX - 1;           // interfaces below the surface
  cplx<double> Ns[NI], Ds[NI];           // projective reflection state below interface l
  constexpr bool kHm = LMAX >= 12;
  constexpr bool kCkpt = LMAX >= 12;     // interface states of even interfaces only
  auto u_of = [&](int l) { return csqrt_fast(cplx<double>{lam2 + k2[l].re, k2[l].im}); };
  auto u_hm = [&](int l, double &hm) { return csqrt_hm(cplx<double>{lam2 + k2[l].re, k2[l].im}, hm); };
  auto half_rcp = [](cplx<double> u, double hm) {   // 1/(2u); hm is unused (dead) unless kHm
    return kHm ? cplx<double>{u.re * hm, -u.im * hm} : crcp_fast(2.0 * u);
  };
  if (L == 1) {
    // r = -k2_0 / (lam + u_0)^2
    double hm0;
    const cplx<double> u0 = u_hm(0, hm0);
    const cplx<double> s = {lam + u0.re, u0.im};
    const cplx<double> D = csq(s);
    const cplx<double> N = {-k2[0].re, -k2[0].im};
    // Im r as the forward model forms it: Im(N conj D) / |D|^2
    const double inv = fast_rcp(D.re * D.re + D.im * D.im);
    imr = (N.im * D.re - N.re * D.im) * inv;
    const cplx<double> iD = {D.re * inv, -D.im * inv};
    const cplx<double> Nb = wt * iD;
    const cplx<double> r = N * iD;
    const cplx<double> Db = {-(Nb * r).re, -(Nb * r).im};
    const cplx<double> ub = Db * (2.0 * s);
    G[0] = G[0] + (ub * half_rcp(u0, hm0) - Nb);
    return;
  }
  // ---- bottom-up: the deepest interface, then step_up through every interface above
  cplx<double> ua = u_of(L - 2);
  cplx<double> N = k2[L - 2] - k2[L - 1], D = csq(ua + u_of(L - 1));
#pragma unroll
  for (int l = NI - 1; l >= 0; --l) {
    if (l <= L - 2) {
      if (l < L - 2) {
        const cplx<double> u = u_of(l);
        const double hh = h2v[l + 1];
        step_up(N, D, u, ua, cexp_tab(cplx<double>{hh * ua.re, hh * ua.im}, phase, e2));
        ua = u;
      }
      if (!kCkpt || (l & 1) == 0) {   // checkpointed: the even interfaces only
        Ns[l] = N;
        Ds[l] = D;
      }
    }
  }
  // surface: a = lam, b = u_0
  const cplx<double> u0 = ua;
  const cplx<double> E0 = cexp_tab(cplx<double>{h2v[0] * u0.re, h2v[0] * u0.im}, phase, e2);
  step_up(N, D, cplx<double>{lam, 0.0}, u0, E0);
  // ---- top-down adjoint
  const double inv = fast_rcp(D.re * D.re + D.im * D.im);
  imr = (N.im * D.re - N.re * D.im) * inv;   // Im r as the forward model forms it
  const cplx<double> iD = {D.re * inv, -D.im * inv};
  const cplx<double> rs = N * iD;        // the reflection coefficient at the surface
  cplx<double> Nb = wt * iD;
  cplx<double> Db = Nb * rs;
  Db = {-Db.re, -Db.im};
  cplx<double> uab;                      // adjoint of u of the layer above the interface
  {
    const cplx<double> NE = Ns[0] * E0;
    const cplx<double> T = Ds[0] - NE;
    const cplx<double> Pb = Nb + Db, Qb = Db - Nb;
    const cplx<double> Sb = lam * Pb, Tb = Qb * u0;
    uab = Qb * T;
    Db = Sb + Tb;
    const cplx<double> NEb = Sb - Tb;
    Nb = NEb * E0;
    const cplx<double> EbE = (NEb * Ns[0]) * E0;
    uab = uab + h2v[0] * EbE;
    H[0] += -2.0 * (EbE * u0).im;
  }
  ua = u0;
  double hma = 0.5 * fast_rcp(u0.re * u0.re + u0.im * u0.im);   // 1/(2|u_l|^2) (kHm)
  // checkpointed: u, 1/(2|u|^2) and E of the layer below an odd interface, formed while
  // rebuilding that interface's state and taken over by the next step
  cplx<double> cu = {0.0, 0.0}, cE = {0.0, 0.0};
  double chm = 0.0;
#pragma unroll
  for (int l = 0; l < NI - 1; ++l) {
    if (l < L - 2) {
      // the step that made state l from state l + 1: a = u_l, b = u_{l+1}, E_{l+1}
      double hmb;
      cplx<double> ub, E;
      const double hh = h2v[l + 1];
      if (kCkpt && (l & 1)) {
        ub = cu;
        hmb = chm;
        E = cE;
      } else {
        ub = u_hm(l + 1, hmb);
        E = cexp_tab(cplx<double>{hh * ub.re, hh * ub.im}, phase, e2);
      }
      cplx<double> N1, D1;               // the state below interface l + 1
      if (!kCkpt || ((l + 1) & 1) == 0) {
        N1 = Ns[l + 1];
        D1 = Ds[l + 1];
      } else {
        cu = u_hm(l + 2, chm);
        if (l + 1 < L - 2) {             // one step up from the stored state below
          const double h2 = h2v[l + 2];
          cE = cexp_tab(cplx<double>{h2 * cu.re, h2 * cu.im}, phase, e2);
          N1 = Ns[l + 2];
          D1 = Ds[l + 2];
          step_up(N1, D1, ub, cu, cE);
        } else {                         // the deepest interface
          N1 = k2[l + 1] - k2[l + 2];
          D1 = csq(ub + cu);
        }
      }
      const cplx<double> NE = N1 * E;
      const cplx<double> S = D1 + NE, T = D1 - NE;
      const cplx<double> Pb = Nb + Db, Qb = Db - Nb;
      uab = uab + Pb * S;
      G[l] = G[l] + uab * half_rcp(ua, hma);                       // u_l complete
      const cplx<double> Sb = Pb * ua, Tb = Qb * ub;
      Db = Sb + Tb;
      const cplx<double> NEb = Sb - Tb;
      Nb = NEb * E;
      const cplx<double> EbE = (NEb * N1) * E;
      uab = Qb * T + hh * EbE;
      H[l + 1] += -2.0 * (EbE * ub).im;
      ua = ub;
      hma = hmb;
    }
  }
  // the deepest interface: N = k2_{L-2} - k2_{L-1}, D = (u_{L-2} + u_{L-1})^2
  double hml;
  cplx<double> ul;
  if (kCkpt && (L & 1)) {                // L - 2 odd: formed with the deepest state
    ul = cu;
    hml = chm;
  } else {
    ul = u_hm(L - 1, hml);
  }
  const cplx<double> sb = Db * (2.0 * (ua + ul));
  const cplx<double> g0 = Nb + (uab + sb) * half_rcp(ua, hma), g1 = sb * half_rcp(ul, hml) - Nb;
#pragma unroll
  for (int l = 0; l < NI; ++l)       // compile-time indices keep G in registers
    if (l == L - 2) {
      G[l] = G[l] + g0;
      G[l + 1] = G[l + 1] + g1;
    }
}

// Single pass.  The reverse sweep of a (lam, w) pair is linear in its seed, and the
// pair's bottom-up recursion already gives Im r_TE, so every pair is visited once: the
// sweep is seeded with the filter coefficient c_k alone, giving per frequency the
// derivatives of Im H(w_j) with respect to the layer wavenumbers and thicknesses; these
// are mapped through the Cole-Cole terms to a per-frequency slot vector u_j, and
// Im H(w_j) is summed on the way.  Once the likelihood is known, the gradient is
// sum_j wbar_j u_j with wbar_j = d ll / d Im H(w_j) = sum_g K_gj ybar_g.  The 4- and
// 8-layer instantiations park every u_j in LDS and form wbar; the 12- and 16-layer ones
// fold each round's eight u_j into V_g = sum_j K_gj u_j (the gradient is then
// sum_g ybar_g V_g), which for fewer gates than frequencies takes less LDS: with 20 gates
// and 40 frequencies a 16-layer workgroup needs 39 KB instead of 52, so four of them (two
// waves per SIMD) fit a compute unit's 160 KB instead of three.  K is read from global
// memory (L2; the fold's K_gj are wave-uniform).
template <int LMAX>
struct AdjShared1 {
  double omega[kMaxFreq], eps2[kMaxGate];
  cplx<double> phase[kPhaseN];
  double exp2t[kExp2N];
  LayerStack stack[kWavesA];
  double imh[kWavesA][kMaxFreq];   // Im H(w_j), then wbar_j (4 and 8 layers)
  double ybar[kWavesA][kMaxGate];
  cplx<double> k2[kWavesA][8][LMAX];
  double h2[kWavesA][kMaxLayers];
  double gl[kWavesA][3 * LMAX + 2];
  double ll[kWavesA];
};

// perm != nullptr: slot j evaluates particle perm[j] for the slots from *first (0 when
// first is NULL) up to *last (device counters of the capacity sort); otherwise slot j is
// particle j (workgroups renumbered XCD-contiguous).
template <int LMAX>
// The 12- and 16-layer instantiations are held to two waves per SIMD: some registers
// spill to private memory (160 and 320 bytes per lane, with the checkpointed interface
// states; 192 and 408 with every state kept), and both still run faster than at one wave
// per SIMD without spills.  The 8-layer one fits two waves without spills
// unconstrained; the same attribute on it (the allocation differs) was 6% slower, and
// held to three waves per SIMD (320 bytes of spills) 5% slower.
__global__ __launch_bounds__(kWave * kWavesA) __attribute__((amdgpu_waves_per_eu(LMAX >= 12 ? 2 : 1))) void loglik_grad1_kernel(DevSystem s, DevParticles p, int kc, int km,
                                                                        const double *y_obs, double *ll, DevGrad g,
                                                                        const int32_t *perm, const int *first,
                                                                        const int *last) {
  __shared__ AdjShared1<LMAX> sm;
  constexpr int NS = 3 * LMAX + 2;
  constexpr bool kByGate = LMAX >= 12;
  // dynamic: the filter's abscissae and coefficients [2][n_hankel_pad], then per wave
  // u_j [n_freq][NS] (4 and 8 layers) or V [n_gate][NS] and the round's u_j [8][NS]
  extern __shared__ double su[];
  const int nf = s.n_freq, ng = s.n_gate, nhp = s.n_hankel_pad;
  double *lam_s = su, *ck_s = su + nhp;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  int64_t i;
  if (perm) {
    const int64_t lo = first ? *first : 0, hi = *last;
    const int64_t slot = lo + (int64_t)blockIdx.x * kWavesA + wave;
    i = slot < hi && slot < p.n ? (int64_t)perm[slot] : p.n;
  } else {
    i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kWavesA + wave;
  }
  const bool valid = i < p.n;
  const bool skip = valid && p.mask && p.mask[i] != p.mask_value;   // left untouched
  if (!__syncthreads_or(valid && !skip)) return;
  for (int t = threadIdx.x; t < nhp; t += blockDim.x) {
    lam_s[t] = s.lam[t];
    ck_s[t] = s.ck[t];
  }
  for (int t = threadIdx.x; t < nf; t += blockDim.x) sm.omega[t] = s.omega[t];
  for (int t = threadIdx.x; t < ng; t += blockDim.x) sm.eps2[t] = s.eps_an2[t];
  for (int t = threadIdx.x; t < kPhaseN; t += blockDim.x)
    sm.phase[t] = cplx<double>{s.phase[2 * t], s.phase[2 * t + 1]};
  for (int t = threadIdx.x; t < kExp2N; t += blockDim.x) sm.exp2t[t] = s.exp2t[t];
  LayerStack *st = &sm.stack[wave];
  double *uw = su + 2 * (size_t)nhp + (size_t)wave * (kByGate ? ng + 8 : nf) * NS;
  double *vw = uw;   // V (kByGate)
  if (kByGate) {
    uw += (size_t)ng * NS;
    for (int t = lane; t < ng * NS; t += kWave) vw[t] = 0.0;
  }
  __syncthreads();
  const int L = merge_particle(p, i, valid && !skip, kc, km, LMAX, st, s.flags);
  double c = 0.0, log_tau = 0.0, spc = 0.0, cpc = 1.0;
  if (L > 0) {
    c = p.c[i];
    log_tau = p.log10_tau[i] * kLn10;
    sincospi(0.5 * c, &spc, &cpc);
    if (lane < L - 1) sm.h2[wave][lane] = -2.0 * (st->top[lane + 1] - st->top[lane]);
  }
  const int gl = lane & 7, gw = lane >> 3;
  const int nhg = nhp >> 3;
  const int nq = (nf + 7) >> 3;
#pragma unroll 1
  for (int q = 0; q < nq; ++q) {
    const int jf = gw + 8 * q;
    const bool act = L > 0 && jf < nf;
    cplx<double> qcc = {0.0, 0.0}, zc = {0.0, 0.0};
    double w = 0.0;
    if (act) {
      w = sm.omega[jf];
      const double pw = exp(c * (log(w) + log_tau));
      zc = cplx<double>{pw * cpc, pw * spc};
      qcc = crcp(cplx<double>{1.0 + zc.re, zc.im});
      const double wmu = w * kMu0A;
      for (int l = gl; l < L; l += 8) {
        const double sg = st->sig[l], mg = st->m[l];
        const cplx<double> sh = {sg * (1.0 - mg * qcc.re), sg * (-(mg * qcc.im))};
        sm.k2[wave][gw][l] = cplx<double>{-(wmu * sh.im), wmu * sh.re};
      }
    }
    wave_lds_sync();
    if (act) {
      cplx<double> G[LMAX];
      double H[LMAX];
#pragma unroll
      for (int l = 0; l < LMAX; ++l) {
        G[l] = {0.0, 0.0};
        H[l] = 0.0;
      }
      double acc = 0.0;
#pragma unroll 1
      for (int sidx = 0; sidx < nhg; ++sidx) {
        const int k = gl + 8 * sidx;
        double imr;
        pair_adjoint<LMAX>(lam_s[k], sm.k2[wave][gw], sm.h2[wave], L, ck_s[k], G, H, sm.phase, sm.exp2t, imr);
        acc = __builtin_fma(ck_s[k], imr, acc);
      }
      acc += __shfl_xor(acc, 1);
      acc += __shfl_xor(acc, 2);
      acc += __shfl_xor(acc, 4);
#pragma unroll
      for (int l = 0; l < LMAX; ++l) {
#pragma unroll
        for (int o = 1; o < 8; o <<= 1) {
          G[l].re += __shfl_xor(G[l].re, o);
          G[l].im += __shfl_xor(G[l].im, o);
          H[l] += __shfl_xor(H[l], o);
        }
      }
      if (gl == 0) {
        sm.imh[wave][jf] = acc;
        // Cole-Cole chain of this frequency: k2 = i w mu0 sigma (1 - m q), q = 1/(1 + z),
        // z = (i w tau)^c; slot vector [log10 sigma (LMAX)][m (LMAX)][thickness (LMAX)][tau][c]
        const cplx<double> iwm = {0.0, w * kMu0A};
        cplx<double> Gq = {0.0, 0.0};
        double *sl = uw + (size_t)(kByGate ? gw : jf) * NS;
#pragma unroll
        for (int l = 0; l < LMAX; ++l) {
          double a0 = 0.0, a1 = 0.0, a2 = 0.0;
          if (l < L) {
            const double sg = st->sig[l], mg = st->m[l];
            const cplx<double> dsig = iwm * (cplx<double>{1.0, 0.0} - mg * qcc);
            a0 = (G[l] * dsig).im * kLn10 * sg;
            a1 = (G[l] * (iwm * (-sg * qcc))).im;
            Gq = Gq + G[l] * (iwm * cplx<double>{-sg * mg, 0.0});
            a2 = H[l];
          }
          sl[l] = a0;
          sl[LMAX + l] = a1;
          sl[2 * LMAX + l] = a2;
        }
        const cplx<double> Gz = Gq * cplx<double>{-(csq(qcc)).re, -(csq(qcc)).im};
        sl[3 * LMAX] = (Gz * (c * kLn10 * zc)).im;
        sl[3 * LMAX + 1] = (Gz * (zc * cplx<double>{log(w) + log_tau, kHalfPi})).im;
      }
    }
    wave_lds_sync();
    if constexpr (kByGate) {
      // fold the round's u_j into V: lane t owns slot t of every gate's row; the round's
      // frequencies are added in order
      if (L > 0 && lane < NS) {
        const int nj = min(8, nf - 8 * q);
        double uv[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) uv[r] = r < nj ? uw[r * NS + lane] : 0.0;
        for (int gg = 0; gg < ng; ++gg) {
          const double *kr = s.K + (size_t)gg * nf + 8 * q;
          double a = vw[gg * NS + lane];
#pragma unroll
          for (int r = 0; r < 8; ++r)
            if (r < nj) a = fma(kr[r], uv[r], a);
          vw[gg * NS + lane] = a;
        }
      }
      wave_lds_sync();
    }
  }
  // gates, the log-likelihood and ybar_g = d ll / d y_g
  if (L > 0) {
    double term = 0.0;
    if (lane < ng) {
      double y = 0.0;
      for (int j = 0; j < nf; ++j) y += s.K[lane * nf + j] * sm.imh[wave][j];
      const int64_t snd = p.n_per_sounding > 0 ? i / p.n_per_sounding : 0;
      const double d = y_obs[snd * ng + lane];
      const double e = s.eps_mn * y;
      const double s2 = sm.eps2[lane] + e * e;
      const double r = d - y;
      term = r * r / s2 + log(kTwoPiA * s2);
      sm.ybar[wave][lane] = r / s2 + (r * r / (s2 * s2) - 1.0 / s2) * s.eps_mn * s.eps_mn * y;
    }
    term += __shfl_xor(term, 1);
    term += __shfl_xor(term, 2);
    term += __shfl_xor(term, 4);
    term += __shfl_xor(term, 8);
    term += __shfl_xor(term, 16);
    term += __shfl_xor(term, 32);
    if (lane == 0) sm.ll[wave] = -0.5 * term;
  }
  wave_lds_sync();
  if constexpr (kByGate) {
    if (L > 0) {
      for (int t = lane; t < NS; t += kWave) {
        double acc = 0.0;
        for (int gg = 0; gg < ng; ++gg) acc += sm.ybar[wave][gg] * vw[(size_t)gg * NS + t];
        sm.gl[wave][t] = acc;
      }
    }
  } else {
    // wbar_j overwrites Im H(w_j), which every gate has read before the last sync
    if (L > 0 && lane < nf) {
      double acc = 0.0;
      for (int gg = 0; gg < ng; ++gg) acc += s.K[gg * nf + lane] * sm.ybar[wave][gg];
      sm.imh[wave][lane] = acc;
    }
    wave_lds_sync();
    if (L > 0) {
      for (int t = lane; t < NS; t += kWave) {
        double acc = 0.0;
        for (int j = 0; j < nf; ++j) acc += sm.imh[wave][j] * uw[(size_t)j * NS + t];
        sm.gl[wave][t] = acc;
      }
    }
  }
  wave_lds_sync();
  if (valid && !skip && lane == 0) {
    const int64_t S = p.stride;
    const bool dec = p.layout == RJSMC_LAYOUT_DECOUPLED;
    const int rows_m = dec ? km : kc + 1;
    g.phi_b[i] = 0.0;
    g.log10_tau[i] = L > 0 ? sm.gl[wave][3 * LMAX] : 0.0;
    g.c[i] = L > 0 ? sm.gl[wave][3 * LMAX + 1] : 0.0;
    for (int r = 0; r < kc; ++r) {
      g.phi[r * S + i] = 0.0;
      g.z_cond[r * S + i] = 0.0;
    }
    for (int r = 0; r < rows_m; ++r) g.m[r * S + i] = 0.0;
    if (dec)
      for (int r = 0; r < km; ++r) g.z_charg[r * S + i] = 0.0;
    double llv = -HUGE_VAL;
    if (L > 0) {
      const double *gv = sm.gl[wave];
      for (int l = 0; l < L; ++l) {
        const int ss = st->src_sig[l];
        if (ss < 0)
          g.phi_b[i] += gv[l];
        else
          g.phi[ss * S + i] += gv[l];
        const int sm_ = st->src_m[l];
        if (sm_ >= 0) g.m[sm_ * S + i] += gv[LMAX + l];
        if (l >= 1) {
          const double dz = gv[2 * LMAX + l - 1] - (l <= L - 2 ? gv[2 * LMAX + l] : 0.0);
          const int src = st->src_top[l];
          if (src >= kMaxLayers)
            g.z_charg[(src - kMaxLayers) * S + i] += dz;
          else
            g.z_cond[src * S + i] += dz;
        }
      }
      llv = sm.ll[wave];
      if (llv != llv) llv = -HUGE_VAL;
    }
    ll[i] = llv;
  }
}

template <int LMAX>
static hipError_t launch_g1(const DevSystem &s, const DevParticles &p, int kc, int km, const double *y_obs,
                            double *ll, const DevGrad &g, hipStream_t stream, const int32_t *perm, const int *first,
                            const int *last) {
  const int64_t blocks = (p.n + kWavesA - 1) / kWavesA;   // every slot range fits
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const size_t per_wave = LMAX >= 12 ? s.n_gate + 8 : s.n_freq;   // slot-vector rows
  const size_t dyn = sizeof(double) * (2 * (size_t)s.n_hankel_pad + kWavesA * per_wave * (3 * LMAX + 2));
  hipLaunchKernelGGL((loglik_grad1_kernel<LMAX>), dim3((unsigned)blocks), dim3(kWave * kWavesA), dyn, stream, s, p,
                     kc, km, y_obs, ll, g, perm, first, last);
  return hipGetLastError();
}

// Particles are evaluated by the instantiation whose layer capacity covers them: with
// a workspace for an evaluation order (ws) and more than 8 layers of capacity, the
// particles are ordered by descending capacity kappa + lambda + 1 on the device (the
// counting sort of the forward's tile shapes); those above 12 layers go to the 16-layer
// instantiation, those of 9 to 12 to the 12-layer one and the others to the 8-layer one
// (each unrolled over its own capacity); otherwise one launch of the smallest
// instantiation that covers the context's capacity.
hipError_t launch_loglik_grad(const DevSystem &s, const DevParticles &p, int kc, int km, const double *y_obs,
                              double *ll, const DevGrad &g, hipStream_t stream, const MutateWorkspace *ws) {
  const int lcap = p.layout == RJSMC_LAYOUT_DECOUPLED ? kc + km + 1 : kc + 1;
  if (lcap <= 4) return launch_g1<4>(s, p, kc, km, y_obs, ll, g, stream, nullptr, nullptr, nullptr);
  if (lcap <= 8) return launch_g1<8>(s, p, kc, km, y_obs, ll, g, stream, nullptr, nullptr, nullptr);
  if (!ws || !ws->perm || p.n > ws->n || p.n < kBucketMin) {
    if (lcap <= 12) return launch_g1<12>(s, p, kc, km, y_obs, ll, g, stream, nullptr, nullptr, nullptr);
    return launch_g1<16>(s, p, kc, km, y_obs, ll, g, stream, nullptr, nullptr, nullptr);
  }
  hipError_t e = launch_layer_sort(p, ws->cnt, ws->perm, stream);
  // after the sort, cnt[kMaxLayers + b] is the end of bin b (bin b: capacity kMaxLayers - b)
  const int *end_13 = ws->cnt + kMaxLayers + (kMaxLayers - 13);   // capacities 16 .. 13
  const int *end_9 = ws->cnt + kMaxLayers + (kMaxLayers - 9);     // capacities 12 .. 9
  const int *end_all = ws->cnt + kMaxLayers + (kMaxLayers - 1);   // every particle
  if (e == hipSuccess && lcap > 12)
    e = launch_g1<16>(s, p, kc, km, y_obs, ll, g, stream, ws->perm, nullptr, end_13);
  if (e == hipSuccess) e = launch_g1<12>(s, p, kc, km, y_obs, ll, g, stream, ws->perm, lcap > 12 ? end_13 : nullptr, end_9);
  if (e == hipSuccess) e = launch_g1<8>(s, p, kc, km, y_obs, ll, g, stream, ws->perm, end_9, end_all);
  return e;
}

}  // namespace rjsmc
