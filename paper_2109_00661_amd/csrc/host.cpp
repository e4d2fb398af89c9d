// Host runtime of librjsmc: context creation, argument validation, error reporting and
// the one-time construction of the frequency-to-time matrix.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rjsmc_internal.h"

namespace {

thread_local std::string g_last_error;

rjsmc_status fail(rjsmc_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
rjsmc_status fail(rjsmc_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

rjsmc_status hip_fail(hipError_t e, const char *what) {
  return fail(e == hipErrorOutOfMemory ? RJSMC_E_NOMEM : RJSMC_E_DEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

// ---------------------------------------------------------------------------------
// Frequency-to-time matrix.
//
// With v_j = Im H(w_j) / w_j and S the natural cubic spline of v in x = ln w, the
// off-time field of a step-off is B(t) = -(2/pi) mu0 F(t) with
//   F(t) = int_{w_0}^{w_{n-1}} S(ln w) cos(w t) dw + v_0 sin(w_0 t)/t - v_{n-1} sin(w_{n-1} t)/t
// (Im H / w held constant below w_0 and above w_{n-1}), and a gate reports
//   y_g = -(2/pi) mu0 1e12 [F(t_open) - F(t_close)] / (t_close - t_open)   [pT/s].
// Everything is linear in Im H, so y = K Im H.  Each spline piece is a cubic in
// (ln w - ln w_m); its products with cos(w t) are integrated by Gauss-Legendre panels
// spanning at most 1.5 rad of phase, in 80-bit long double.
// ---------------------------------------------------------------------------------
typedef long double ld;

void gauss_legendre(int n, std::vector<ld> &x, std::vector<ld> &w) {
  x.assign(n, 0);
  w.assign(n, 0);
  const ld pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    ld z = cosl(pi * (i + 0.75L) / (n + 0.5L));
    for (int it = 0; it < 100; ++it) {
      ld p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      ld dp = n * (z * p1 - p0) / (z * z - 1);
      ld dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) {
        // recompute derivative at the converged node
        p0 = 1;
        p1 = z;
        for (int k = 2; k <= n; ++k) {
          ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1);
        x[i] = z;
        w[i] = 2 / ((1 - z * z) * dp * dp);
        break;
      }
    }
  }
}

// mom[p] = int_{wa}^{wb} (ln w - ln wa)^p cos(w t) dw, p = 0..3
void cos_moments(ld wa, ld wb, ld t, const std::vector<ld> &gx, const std::vector<ld> &gw,
                 ld mom[4]) {
  const ld max_phase = 1.5L;
  long npan = (long)ceill((wb - wa) * t / max_phase);
  if (npan < 1) npan = 1;
  const ld xa = logl(wa);
  const ld width = (wb - wa) / npan;
  ld acc[4] = {0, 0, 0, 0};
  for (long k = 0; k < npan; ++k) {
    const ld lo = wa + width * k;
    const ld mid = lo + width / 2, half = width / 2;
    ld pan[4] = {0, 0, 0, 0};
    for (size_t i = 0; i < gx.size(); ++i) {
      const ld om = mid + half * gx[i];
      const ld cw = cosl(om * t) * gw[i];
      const ld s = logl(om) - xa;
      pan[0] += cw;
      pan[1] += cw * s;
      pan[2] += cw * s * s;
      pan[3] += cw * s * s * s;
    }
    for (int p = 0; p < 4; ++p) acc[p] += pan[p] * half;
  }
  for (int p = 0; p < 4; ++p) mom[p] = acc[p];
}

}  // namespace

namespace rjsmc {

void build_time_kernel(const double *freq_hz, int nf, const double *t_open, const double *t_close,
                       int ng, double *K_out) {
  const ld pi = 3.141592653589793238462643383279502884L;
  const ld mu0 = 4e-7L * pi;
  std::vector<ld> w(nf), x(nf), hx(nf - 1);
  for (int i = 0; i < nf; ++i) {
    w[i] = 2 * pi * (ld)freq_hz[i];
    x[i] = logl(w[i]);
  }
  for (int i = 0; i + 1 < nf; ++i) hx[i] = x[i + 1] - x[i];
  std::vector<ld> gx, gw;
  gauss_legendre(20, gx, gw);

  // moments for every gate edge: times[0..ng) = open, [ng..2ng) = close
  std::vector<ld> times(2 * ng);
  for (int g = 0; g < ng; ++g) {
    times[g] = t_open[g];
    times[ng + g] = t_close[g];
  }
  std::vector<ld> mom((size_t)(nf - 1) * 4 * 2 * ng);
  for (int m = 0; m + 1 < nf; ++m)
    for (int it = 0; it < 2 * ng; ++it) {
      ld mm[4];
      cos_moments(w[m], w[m + 1], times[it], gx, gw, mm);
      for (int p = 0; p < 4; ++p) mom[((size_t)m * 4 + p) * 2 * ng + it] = mm[p];
    }

  std::vector<ld> v(nf), M(nf), diag(nf), rhs(nf), F(2 * ng);
  for (int j = 0; j < nf; ++j) {
    for (int i = 0; i < nf; ++i) v[i] = (i == j) ? 1 / w[j] : 0;
    // natural spline second derivatives: Thomas algorithm on rows 1..nf-2
    std::fill(M.begin(), M.end(), 0.0L);
    if (nf > 2) {
      std::vector<ld> cprime(nf, 0), dprime(nf, 0);
      for (int i = 1; i <= nf - 2; ++i) {
        const ld a = hx[i - 1], b = 2 * (hx[i - 1] + hx[i]), c = hx[i];
        const ld d = 6 * ((v[i + 1] - v[i]) / hx[i] - (v[i] - v[i - 1]) / hx[i - 1]);
        const ld den = b - (i > 1 ? a * cprime[i - 1] : 0);
        cprime[i] = c / den;
        dprime[i] = (d - (i > 1 ? a * dprime[i - 1] : 0)) / den;
      }
      for (int i = nf - 2; i >= 1; --i) M[i] = dprime[i] - (i < nf - 2 ? cprime[i] * M[i + 1] : 0);
    }
    for (int it = 0; it < 2 * ng; ++it) {
      const ld t = times[it];
      ld acc = v[0] * sinl(w[0] * t) / t - v[nf - 1] * sinl(w[nf - 1] * t) / t;
      for (int m = 0; m + 1 < nf; ++m) {
        const ld h = hx[m];
        const ld a0 = v[m];
        const ld a1 = (v[m + 1] - v[m]) / h - h * (2 * M[m] + M[m + 1]) / 6;
        const ld a2 = M[m] / 2;
        const ld a3 = (M[m + 1] - M[m]) / (6 * h);
        const ld *mo = &mom[(size_t)m * 4 * 2 * ng];
        acc += a0 * mo[0 * 2 * ng + it] + a1 * mo[1 * 2 * ng + it] + a2 * mo[2 * 2 * ng + it] +
               a3 * mo[3 * 2 * ng + it];
      }
      F[it] = acc;
    }
    for (int g = 0; g < ng; ++g) {
      const ld y = -(2 / pi) * mu0 * 1e12L * (F[g] - F[ng + g]) / (times[ng + g] - times[g]);
      K_out[(size_t)g * nf + j] = (double)y;
    }
  }
}

}  // namespace rjsmc

// ---------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------
using rjsmc::DevParticles;

extern "C" const char *rjsmc_last_error(void) { return g_last_error.c_str(); }

static void free_dev(rjsmc::DevSystem &d) {
  void *ptrs[] = {d.omega, d.lam, d.ck, d.K, d.eps_an2, d.phase, d.exp2t, d.flags};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  memset(&d, 0, sizeof d);
}

extern "C" rjsmc_status rjsmc_create(const rjsmc_system *s, int device, rjsmc_ctx **out) {
  if (!s || !out) return fail(RJSMC_E_INVALID, "rjsmc_create: NULL argument");
  *out = nullptr;
  if (s->n_freq < 2 || s->n_freq > rjsmc::kMaxFreq)
    return fail(RJSMC_E_INVALID, "rjsmc_create: n_freq=%d outside 2..%d", s->n_freq, rjsmc::kMaxFreq);
  if (s->n_hankel < 1 || s->n_hankel > rjsmc::kMaxHankel)
    return fail(RJSMC_E_INVALID, "rjsmc_create: n_hankel=%d outside 1..%d", s->n_hankel,
                rjsmc::kMaxHankel);
  if (s->n_gate < 1 || s->n_gate > rjsmc::kMaxGate)
    return fail(RJSMC_E_INVALID, "rjsmc_create: n_gate=%d outside 1..%d", s->n_gate, rjsmc::kMaxGate);
  if (!s->freq_hz || !s->hankel_b || !s->hankel_w || !s->gate_open_s || !s->gate_close_s || !s->eps_an)
    return fail(RJSMC_E_INVALID, "rjsmc_create: NULL table pointer");
  if (s->kmax_cond < 0 || s->kmax_charg < 0 || s->kmax_cond + s->kmax_charg + 1 > rjsmc::kMaxLayers)
    return fail(RJSMC_E_INVALID, "rjsmc_create: capacities %d+%d+1 exceed %d layers", s->kmax_cond,
                s->kmax_charg, rjsmc::kMaxLayers);
  if (s->fwd_precision != RJSMC_F64 && s->fwd_precision != RJSMC_F32)
    return fail(RJSMC_E_INVALID, "rjsmc_create: bad precision %d", s->fwd_precision);
  if (!(s->loop_radius_m > 0) || !(s->height_m >= 0) || !(s->eps_mn >= 0))
    return fail(RJSMC_E_INVALID, "rjsmc_create: bad geometry or noise");
  for (int i = 0; i < s->n_freq; ++i)
    if (!(s->freq_hz[i] > 0) || (i && !(s->freq_hz[i] > s->freq_hz[i - 1])))
      return fail(RJSMC_E_INVALID, "rjsmc_create: frequencies must be positive and increasing");
  for (int g = 0; g < s->n_gate; ++g)
    if (!(s->gate_open_s[g] > 0) || !(s->gate_close_s[g] > s->gate_open_s[g]))
      return fail(RJSMC_E_INVALID, "rjsmc_create: gate %d has bad times", g);

  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_create: hipSetDevice");
  // the address of the device's copy of the static scratch of rjsmc_mutate_noalloc (once
  // per device); a failure is reported by that entry point, the context works without it
  (void)rjsmc::static_scratch_init(device);

  rjsmc_ctx *c = new rjsmc_ctx();
  c->device = device;
  c->kmax_cond = s->kmax_cond;
  c->kmax_charg = s->kmax_charg;
  c->precision = s->fwd_precision;
  c->z_max = s->z_max_m;
  rjsmc::DevSystem &d = c->dev;
  memset(&d, 0, sizeof d);
  d.n_freq = s->n_freq;
  d.n_hankel = s->n_hankel;
  d.n_hankel_pad = (s->n_hankel + 7) / 8 * 8;
  d.n_gate = s->n_gate;
  d.eps_mn = s->eps_mn;

  const int nf = s->n_freq, nh = s->n_hankel, nhp = d.n_hankel_pad, ng = s->n_gate;
  std::vector<double> omega(nf), lam(nhp, 1.0), ck(nhp, 0.0), eps2(ng);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < nf; ++i) omega[i] = 2.0 * pi * s->freq_hz[i];
  for (int k = 0; k < nh; ++k) {
    lam[k] = s->hankel_b[k] / s->loop_radius_m;
    ck[k] = 0.5 * s->current_a * s->hankel_w[k] * lam[k] * std::exp(-2.0 * lam[k] * s->height_m);
  }
  for (int g = 0; g < ng; ++g) eps2[g] = s->eps_an[g] * s->eps_an[g];
  // tables of the propagation-factor exponential, from extended-precision libm
  std::vector<double> phase(2 * rjsmc::kPhaseN), exp2t(rjsmc::kExp2N);
  const long double pil = acosl(-1.0L);
  for (int j = 0; j < rjsmc::kPhaseN; ++j) {
    phase[2 * j] = (double)cosl(pil * j / 128);
    phase[2 * j + 1] = (double)sinl(pil * j / 128);
  }
  for (int j = 0; j < rjsmc::kExp2N; ++j) exp2t[j] = (double)exp2l(j / 256.0L);
  c->K_host = new double[(size_t)ng * nf];
  rjsmc::build_time_kernel(s->freq_hz, nf, s->gate_open_s, s->gate_close_s, ng, c->K_host);

  struct Up {
    double **dst;
    const double *src;
    size_t n;
  } ups[] = {{&d.omega, omega.data(), (size_t)nf},
             {&d.lam, lam.data(), (size_t)nhp},
             {&d.ck, ck.data(), (size_t)nhp},
             {&d.K, c->K_host, (size_t)ng * nf},
             {&d.eps_an2, eps2.data(), (size_t)ng},
             {&d.phase, phase.data(), phase.size()},
             {&d.exp2t, exp2t.data(), exp2t.size()}};
  for (auto &u : ups) {
    e = hipMalloc((void **)u.dst, u.n * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(*u.dst, u.src, u.n * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      free_dev(d);
      delete[] c->K_host;
      delete c;
      return hip_fail(e, "rjsmc_create: table upload");
    }
  }
  e = hipMalloc((void **)&d.flags, sizeof(int));
  if (e == hipSuccess) e = hipMemset(d.flags, 0, sizeof(int));
  c->work_mask = nullptr;
  c->work_type = nullptr;
  c->work_perm = nullptr;
  c->work_cnt = nullptr;
  c->work_gvalid = nullptr;
  c->work_lq = nullptr;
  c->work_rim = nullptr;
  c->work_rim_layers = nullptr;
  c->work_rim_n = 0;
  c->tuning.waves_per_block = 4;
  c->tuning.layer_sort = 0;
  c->tuning.waves_per_particle = 1;
  int lds_limit = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
  c->lds_limit = lds_limit > 0 ? (size_t)lds_limit : 0;
  int n_cu = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
  c->n_cu = n_cu > 0 ? n_cu : 0;
  c->work_n = s->max_particles > 0 ? s->max_particles : 0;
  if (e == hipSuccess && c->work_n > 0) {
    e = hipMalloc((void **)&c->work_mask, sizeof(int32_t) * c->work_n);
    if (e == hipSuccess) e = hipMalloc((void **)&c->work_type, sizeof(int32_t) * c->work_n);
    if (e == hipSuccess) e = hipMalloc((void **)&c->work_perm, sizeof(int32_t) * c->work_n);
    if (e == hipSuccess) e = hipMalloc((void **)&c->work_gvalid, sizeof(int32_t) * c->work_n);
    if (e == hipSuccess) e = hipMalloc((void **)&c->work_lq, sizeof(double) * c->work_n);
    if (e == hipSuccess) e = hipMalloc((void **)&c->work_cnt, sizeof(int) * 2 * rjsmc::kMaxLayers);
    c->work_rim_n = std::min<int64_t>(c->work_n, rjsmc::spread_max_particles());
    if (e == hipSuccess)
      e = hipMalloc((void **)&c->work_rim, sizeof(double) * rjsmc::spread_rim_doubles(d, c->work_rim_n));
    if (e == hipSuccess) e = hipMalloc((void **)&c->work_rim_layers, sizeof(int32_t) * c->work_rim_n);
  }
  if (e != hipSuccess) {
    if (c->work_mask) (void)hipFree(c->work_mask);
    if (c->work_type) (void)hipFree(c->work_type);
    if (c->work_perm) (void)hipFree(c->work_perm);
    if (c->work_cnt) (void)hipFree(c->work_cnt);
    if (c->work_gvalid) (void)hipFree(c->work_gvalid);
    if (c->work_lq) (void)hipFree(c->work_lq);
    if (c->work_rim) (void)hipFree(c->work_rim);
    if (c->work_rim_layers) (void)hipFree(c->work_rim_layers);
    free_dev(d);
    delete[] c->K_host;
    delete c;
    return hip_fail(e, "rjsmc_create: workspace");
  }
  *out = c;
  return RJSMC_OK;
}

extern "C" void rjsmc_destroy(rjsmc_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->work_mask) (void)hipFree(c->work_mask);
  if (c->work_type) (void)hipFree(c->work_type);
  if (c->work_perm) (void)hipFree(c->work_perm);
  if (c->work_cnt) (void)hipFree(c->work_cnt);
  if (c->work_gvalid) (void)hipFree(c->work_gvalid);
  if (c->work_lq) (void)hipFree(c->work_lq);
  if (c->work_rim) (void)hipFree(c->work_rim);
  if (c->work_rim_layers) (void)hipFree(c->work_rim_layers);
  free_dev(c->dev);
  delete[] c->K_host;
  delete c;
}

extern "C" rjsmc_status rjsmc_check(rjsmc_ctx *c, rjsmc_stream stream) {
  if (!c) return fail(RJSMC_E_INVALID, "rjsmc_check: NULL context");
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_check: synchronize");
  int flags = 0;
  e = hipMemcpy(&flags, c->dev.flags, sizeof(int), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemset(c->dev.flags, 0, sizeof(int));
  if (e != hipSuccess) return hip_fail(e, "rjsmc_check: read flags");
  if (flags & rjsmc::kFlagCapacity)
    return fail(RJSMC_E_CAPACITY, "rjsmc_check: a particle exceeded the layer capacity");
  if (flags & rjsmc::kFlagUnsorted)
    return fail(RJSMC_E_INVALID, "rjsmc_check: a particle had unsorted or negative depths");
  return RJSMC_OK;
}

extern "C" rjsmc_status rjsmc_time_kernel(const rjsmc_ctx *c, double *K_out) {
  if (!c || !K_out) return fail(RJSMC_E_INVALID, "rjsmc_time_kernel: NULL argument");
  memcpy(K_out, c->K_host, sizeof(double) * c->dev.n_gate * c->dev.n_freq);
  return RJSMC_OK;
}

extern "C" rjsmc_status rjsmc_build_time_kernel(const double *freq_hz, int32_t nf, const double *t_open,
                                                const double *t_close, int32_t ng, double *K_out) {
  if (!freq_hz || !t_open || !t_close || !K_out)
    return fail(RJSMC_E_INVALID, "rjsmc_build_time_kernel: NULL argument");
  if (nf < 2 || nf > rjsmc::kMaxFreq || ng < 1 || ng > rjsmc::kMaxGate)
    return fail(RJSMC_E_INVALID, "rjsmc_build_time_kernel: bad sizes %d, %d", nf, ng);
  for (int i = 0; i < nf; ++i)
    if (!(freq_hz[i] > 0) || (i && !(freq_hz[i] > freq_hz[i - 1])))
      return fail(RJSMC_E_INVALID, "rjsmc_build_time_kernel: frequencies must be positive and increasing");
  for (int g = 0; g < ng; ++g)
    if (!(t_open[g] > 0) || !(t_close[g] > t_open[g]))
      return fail(RJSMC_E_INVALID, "rjsmc_build_time_kernel: gate %d has bad times", g);
  rjsmc::build_time_kernel(freq_hz, nf, t_open, t_close, ng, K_out);
  return RJSMC_OK;
}

static rjsmc_status check_particles(const rjsmc_ctx *c, const rjsmc_particles *p, const char *who,
                                    DevParticles *dp) {
  if (!p) return fail(RJSMC_E_INVALID, "%s: NULL particles", who);
  if (p->n <= 0) return fail(RJSMC_E_INVALID, "%s: n=%lld must be positive", who, (long long)p->n);
  if (p->stride < p->n)
    return fail(RJSMC_E_INVALID, "%s: stride=%lld < n=%lld", who, (long long)p->stride, (long long)p->n);
  if (p->n_per_sounding < 0) return fail(RJSMC_E_INVALID, "%s: negative n_per_sounding", who);
  if (p->layout != RJSMC_LAYOUT_DECOUPLED && p->layout != RJSMC_LAYOUT_MERGED)
    return fail(RJSMC_E_INVALID, "%s: bad layout %d", who, p->layout);
  const bool dec = p->layout == RJSMC_LAYOUT_DECOUPLED;
  if (!p->kappa || !p->phi_b || !p->log10_tau || !p->c || (c->kmax_cond && (!p->phi || !p->z_cond)) ||
      !p->m || (dec && !p->lambda) || (dec && c->kmax_charg && !p->z_charg))
    return fail(RJSMC_E_INVALID, "%s: NULL particle array", who);
  if (dec && c->kmax_charg == 0 && p->m == nullptr) return fail(RJSMC_E_INVALID, "%s: NULL m", who);
  dp->n = p->n;
  dp->stride = p->stride;
  dp->n_per_sounding = p->n_per_sounding;
  dp->layout = p->layout;
  dp->kappa = p->kappa;
  dp->lambda = p->lambda;
  dp->phi_b = p->phi_b;
  dp->phi = p->phi;
  dp->z_cond = p->z_cond;
  dp->m = p->m;
  dp->z_charg = p->z_charg;
  dp->log10_tau = p->log10_tau;
  dp->c = p->c;
  dp->mask = nullptr;
  return RJSMC_OK;
}

// The context's own workspace (empty when it was created with max_particles = 0).
static rjsmc::MutateWorkspace ctx_workspace(const rjsmc_ctx *c) {
  rjsmc::MutateWorkspace w;
  w.mask = c->work_mask;
  w.type = c->work_type;
  w.gvalid = c->work_gvalid;
  w.perm = c->work_perm;
  w.cnt = c->work_cnt;
  w.lq = c->work_lq;
  w.n = c->work_perm ? c->work_n : 0;
  w.rim = c->work_rim;
  w.rim_layers = c->work_rim_layers;
  w.rim_n = c->work_rim ? c->work_rim_n : 0;
  return w;
}

// Tile shape of a forward launch over dp from the context's tuning; a layer-capacity
// order is computed first (on the same stream) when the tuning asks for one and the
// workspace holds dp.n particles.
static hipError_t forward_tiles(const rjsmc_ctx *c, const rjsmc::DevParticles &dp, const rjsmc_tuning &t,
                                const rjsmc::MutateWorkspace &ws, hipStream_t stream, rjsmc::ForwardTiles *tiles) {
  tiles->waves_per_block = t.waves_per_block;
  tiles->waves_per_particle = t.waves_per_particle;
  tiles->perm = nullptr;
  tiles->n_cu = c->n_cu;
  tiles->rim = ws.rim;
  tiles->rim_layers = ws.rim_layers;
  tiles->rim_n = ws.rim ? ws.rim_n : 0;
  if (t.layer_sort && ws.perm && dp.n <= ws.n && dp.n > 0) {
    const hipError_t e = rjsmc::launch_layer_sort(dp, ws.cnt, ws.perm, stream);
    if (e != hipSuccess) return e;
    tiles->perm = ws.perm;
  }
  return hipSuccess;
}

static hipError_t run_forward(const rjsmc_ctx *c, const rjsmc::DevParticles &dp, const rjsmc_tuning &t, double *resp,
                              const double *y_obs, double *ll, hipStream_t stream,
                              const rjsmc::MutateWorkspace *ws = nullptr) {
  rjsmc::ForwardTiles tiles;
  hipError_t e = forward_tiles(c, dp, t, ws ? *ws : ctx_workspace(c), stream, &tiles);
  if (e == hipSuccess)
    e = rjsmc::launch_forward(c->dev, dp, c->kmax_cond, c->kmax_charg, c->precision, resp, y_obs, ll, stream, tiles);
  return e;
}

extern "C" rjsmc_status rjsmc_forward(rjsmc_ctx *c, const rjsmc_particles *p, double *resp,
                                      rjsmc_stream stream) {
  if (!c) return fail(RJSMC_E_INVALID, "rjsmc_forward: NULL context");
  DevParticles dp;
  rjsmc_status st = check_particles(c, p, "rjsmc_forward", &dp);
  if (st != RJSMC_OK) return st;
  if (!resp) return fail(RJSMC_E_INVALID, "rjsmc_forward: NULL resp");
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess)
    e = run_forward(c, dp, c->tuning, resp, nullptr, nullptr, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_forward: launch");
  return RJSMC_OK;
}

extern "C" rjsmc_status rjsmc_loglik(rjsmc_ctx *c, const rjsmc_particles *p, const double *y_obs,
                                     double *ll, rjsmc_stream stream) {
  if (!c) return fail(RJSMC_E_INVALID, "rjsmc_loglik: NULL context");
  DevParticles dp;
  rjsmc_status st = check_particles(c, p, "rjsmc_loglik", &dp);
  if (st != RJSMC_OK) return st;
  if (!y_obs || !ll) return fail(RJSMC_E_INVALID, "rjsmc_loglik: NULL y_obs or ll");
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess)
    e = run_forward(c, dp, c->tuning, nullptr, y_obs, ll, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_loglik: launch");
  return RJSMC_OK;
}

extern "C" rjsmc_status rjsmc_loglik_grad(rjsmc_ctx *c, const rjsmc_particles *p, const double *y_obs,
                                          double *ll, rjsmc_particles *grad, rjsmc_stream stream) {
  if (!c) return fail(RJSMC_E_INVALID, "rjsmc_loglik_grad: NULL context");
  if (c->precision != RJSMC_F64)
    return fail(RJSMC_E_UNSUPPORTED, "rjsmc_loglik_grad: the adjoint runs in FP64 contexts only");
  DevParticles dp;
  rjsmc_status st = check_particles(c, p, "rjsmc_loglik_grad", &dp);
  if (st != RJSMC_OK) return st;
  if (!y_obs || !ll || !grad) return fail(RJSMC_E_INVALID, "rjsmc_loglik_grad: NULL argument");
  const bool dec = p->layout == RJSMC_LAYOUT_DECOUPLED;
  if (!grad->phi_b || !grad->log10_tau || !grad->c || !grad->m || (c->kmax_cond && (!grad->phi || !grad->z_cond)) ||
      (dec && c->kmax_charg && !grad->z_charg))
    return fail(RJSMC_E_INVALID, "rjsmc_loglik_grad: NULL gradient array");
  rjsmc::DevGrad g{grad->phi_b, grad->phi, grad->z_cond, grad->m, grad->z_charg, grad->log10_tau, grad->c};
  const rjsmc::MutateWorkspace ws = ctx_workspace(c);   // the evaluation order, when it holds n
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess)
    e = rjsmc::launch_loglik_grad(c->dev, dp, c->kmax_cond, c->kmax_charg, y_obs, ll, g, (hipStream_t)stream,
                                  &ws);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_loglik_grad: launch");
  return RJSMC_OK;
}

// ---------------------------------------------------------------------------------
// SMC entry points
// ---------------------------------------------------------------------------------
static rjsmc::SmcShape smc_shape(const rjsmc_ctx *c) {
  rjsmc::SmcShape sh;
  sh.kc = c->kmax_cond;
  sh.km = c->kmax_charg;
  sh.n_models = (c->kmax_cond + 1) * (c->kmax_charg + 1);
  sh.dmax = 3 + 2 * c->kmax_cond + 2 * c->kmax_charg;
  sh.z_max = c->z_max;
  return sh;
}

static rjsmc::DevParticlesW writable(const rjsmc::DevParticles &d) {
  rjsmc::DevParticlesW w;
  w.n = d.n;
  w.stride = d.stride;
  w.n_per_sounding = d.n_per_sounding;
  w.layout = d.layout;
  w.kappa = const_cast<int32_t *>(d.kappa);
  w.lambda = const_cast<int32_t *>(d.lambda);
  w.phi_b = const_cast<double *>(d.phi_b);
  w.phi = const_cast<double *>(d.phi);
  w.z_cond = const_cast<double *>(d.z_cond);
  w.m = const_cast<double *>(d.m);
  w.z_charg = const_cast<double *>(d.z_charg);
  w.log10_tau = const_cast<double *>(d.log10_tau);
  w.c = const_cast<double *>(d.c);
  return w;
}

static rjsmc_status check_prior(const rjsmc_prior *pr, const char *who) {
  if (!pr) return fail(RJSMC_E_INVALID, "%s: NULL prior", who);
  if (!(pr->phi_lo < pr->phi_hi) || !(pr->m_lo < pr->m_hi) || !(pr->ltau_lo < pr->ltau_hi) ||
      !(pr->c_lo < pr->c_hi) || !(pr->m_lo >= 0) || !(pr->m_hi < 1))
    return fail(RJSMC_E_INVALID, "%s: bad prior bounds", who);
  return RJSMC_OK;
}

// Soundings of a population: n_sound * n_per_sounding == n.
static rjsmc_status check_soundings(const rjsmc_particles *p, int32_t n_sound, const char *who) {
  const int64_t nps = p->n_per_sounding > 0 ? p->n_per_sounding : p->n;
  if (n_sound < 1 || nps * (int64_t)n_sound != p->n)
    return fail(RJSMC_E_INVALID, "%s: n_sound=%d does not tile n=%lld", who, n_sound, (long long)p->n);
  if (nps > RJSMC_MAX_PER_SOUNDING)
    return fail(RJSMC_E_UNSUPPORTED, "%s: %lld particles per sounding exceed %d", who, (long long)nps,
                RJSMC_MAX_PER_SOUNDING);
  return RJSMC_OK;
}

extern "C" rjsmc_status rjsmc_init_prior(rjsmc_ctx *c, rjsmc_particles *p, const rjsmc_prior *prior, uint64_t seed,
                                         rjsmc_stream stream) {
  if (!c) return fail(RJSMC_E_INVALID, "rjsmc_init_prior: NULL context");
  rjsmc::DevParticles dp;
  rjsmc_status st = check_particles(c, p, "rjsmc_init_prior", &dp);
  if (st != RJSMC_OK) return st;
  if (p->layout != RJSMC_LAYOUT_DECOUPLED) return fail(RJSMC_E_INVALID, "rjsmc_init_prior: DECOUPLED layout only");
  if ((st = check_prior(prior, "rjsmc_init_prior")) != RJSMC_OK) return st;
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = rjsmc::launch_init_prior(writable(dp), smc_shape(c), *prior, seed, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_init_prior: launch");
  return RJSMC_OK;
}

extern "C" rjsmc_status rjsmc_reweight_resample(rjsmc_ctx *c, const rjsmc_reweight_args *a, const rjsmc_particles *in,
                                                const double *ll_in, rjsmc_particles *out, double *ll_out,
                                                double *gamma, double *log_z, int32_t *active, int32_t *anc,
                                                rjsmc_stream stream) {
  const char *who = "rjsmc_reweight_resample";
  if (!c || !a) return fail(RJSMC_E_INVALID, "%s: NULL argument", who);
  rjsmc::DevParticles di, dout;
  rjsmc_status st = check_particles(c, in, who, &di);
  if (st == RJSMC_OK) st = check_particles(c, out, who, &dout);
  if (st != RJSMC_OK) return st;
  if (in->layout != out->layout || in->n != out->n || in->n_per_sounding != out->n_per_sounding)
    return fail(RJSMC_E_INVALID, "%s: in and out populations differ in shape", who);
  if (in->layout != RJSMC_LAYOUT_DECOUPLED) return fail(RJSMC_E_INVALID, "%s: DECOUPLED layout only", who);
  if (in->kappa == out->kappa || in->phi_b == out->phi_b) return fail(RJSMC_E_INVALID, "%s: out aliases in", who);
  if (!ll_in || !ll_out || !gamma || !log_z || !anc) return fail(RJSMC_E_INVALID, "%s: NULL array", who);
  if (!(a->alpha_tess > 0 && a->alpha_tess < 1)) return fail(RJSMC_E_INVALID, "%s: alpha must be in (0,1)", who);
  if ((st = check_soundings(in, a->n_sound, who)) != RJSMC_OK) return st;
  const rjsmc::SmcShape sh = smc_shape(c);
  if (sh.n_models > 128) return fail(RJSMC_E_UNSUPPORTED, "%s: %d models exceed 128", who, sh.n_models);
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess)
    e = rjsmc::launch_reweight_resample(sh, *a, di, ll_in, writable(dout), ll_out, gamma, log_z, active, anc,
                                        c->dev.flags, c->dev.exp2t, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_reweight_resample: launch");
  return RJSMC_OK;
}

extern "C" rjsmc_status rjsmc_adapt(rjsmc_ctx *c, const rjsmc_particles *p, int32_t n_sound, const rjsmc_prior *prior,
                                    double *factors, rjsmc_stream stream) {
  const char *who = "rjsmc_adapt";
  if (!c || !factors) return fail(RJSMC_E_INVALID, "%s: NULL argument", who);
  rjsmc::DevParticles dp;
  rjsmc_status st = check_particles(c, p, who, &dp);
  if (st != RJSMC_OK) return st;
  if (p->layout != RJSMC_LAYOUT_DECOUPLED) return fail(RJSMC_E_INVALID, "%s: DECOUPLED layout only", who);
  if ((st = check_prior(prior, who)) != RJSMC_OK) return st;
  if ((st = check_soundings(p, n_sound, who)) != RJSMC_OK) return st;
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = rjsmc::launch_adapt(smc_shape(c), dp, n_sound, *prior, factors, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_adapt: launch");
  return RJSMC_OK;
}

// Archive of a current population p (n particles): shapes, slots and arrays.
static rjsmc_status check_archive(const rjsmc_ctx *c, const rjsmc_archive *ar, const rjsmc_particles *p,
                                  const char *who, rjsmc::DevParticles *dpop) {
  if (!ar) return fail(RJSMC_E_INVALID, "%s: NULL archive", who);
  if (ar->n_slots < 1 || ar->n_slots > RJSMC_MAX_ARCHIVE)
    return fail(RJSMC_E_INVALID, "%s: n_slots=%d outside 1..%d", who, ar->n_slots, RJSMC_MAX_ARCHIVE);
  if (ar->n_used < 0 || ar->n_used > ar->n_slots)
    return fail(RJSMC_E_INVALID, "%s: n_used=%d outside 0..n_slots", who, ar->n_used);
  const rjsmc_status st = check_particles(c, &ar->pop, who, dpop);
  if (st != RJSMC_OK) return st;
  if (ar->pop.layout != p->layout) return fail(RJSMC_E_INVALID, "%s: archive layout differs", who);
  if (ar->pop.n != (int64_t)ar->n_slots * p->n)
    return fail(RJSMC_E_INVALID, "%s: archive holds %lld particles, not n_slots x %lld", who, (long long)ar->pop.n,
                (long long)p->n);
  if (!ar->ll || !ar->gamma || !ar->log_z) return fail(RJSMC_E_INVALID, "%s: NULL archive array", who);
  return RJSMC_OK;
}

extern "C" rjsmc_status rjsmc_archive_store(rjsmc_ctx *c, const rjsmc_particles *p, const double *ll,
                                            const double *gamma, const double *log_z, int32_t n_sound,
                                            rjsmc_archive *ar, int32_t slot, rjsmc_stream stream) {
  const char *who = "rjsmc_archive_store";
  if (!c || !ll || !gamma || !log_z) return fail(RJSMC_E_INVALID, "%s: NULL argument", who);
  rjsmc::DevParticles dp, dpop;
  rjsmc_status st = check_particles(c, p, who, &dp);
  if (st != RJSMC_OK) return st;
  if (p->layout != RJSMC_LAYOUT_DECOUPLED) return fail(RJSMC_E_INVALID, "%s: DECOUPLED layout only", who);
  if ((st = check_soundings(p, n_sound, who)) != RJSMC_OK) return st;
  if ((st = check_archive(c, ar, p, who, &dpop)) != RJSMC_OK) return st;
  if (slot < 0 || slot >= ar->n_slots) return fail(RJSMC_E_INVALID, "%s: slot %d outside 0..%d", who, slot,
                                                   ar->n_slots - 1);
  const rjsmc::SmcShape sh = smc_shape(c);
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess)
    e = rjsmc::launch_archive_store(dp, ll, gamma, log_z, n_sound, sh.n_models, writable(dpop), ar->ll, ar->gamma,
                                    ar->log_z, slot, c->kmax_cond, c->kmax_charg, c->kmax_charg,
                                    (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_archive_store: launch");
  return RJSMC_OK;
}

extern "C" rjsmc_status rjsmc_adapt_recycled(rjsmc_ctx *c, const rjsmc_particles *p, const double *ll,
                                             const double *gamma, const double *log_z, int32_t n_sound,
                                             const rjsmc_archive *ar, const rjsmc_prior *prior, double *factors,
                                             rjsmc_stream stream) {
  const char *who = "rjsmc_adapt_recycled";
  if (!c || !factors || !ll || !gamma || !log_z) return fail(RJSMC_E_INVALID, "%s: NULL argument", who);
  rjsmc::DevParticles dp, dpop;
  rjsmc_status st = check_particles(c, p, who, &dp);
  if (st != RJSMC_OK) return st;
  if (p->layout != RJSMC_LAYOUT_DECOUPLED) return fail(RJSMC_E_INVALID, "%s: DECOUPLED layout only", who);
  if ((st = check_prior(prior, who)) != RJSMC_OK) return st;
  if ((st = check_soundings(p, n_sound, who)) != RJSMC_OK) return st;
  if ((st = check_archive(c, ar, p, who, &dpop)) != RJSMC_OK) return st;
  rjsmc::ArchiveView av;
  av.pop = dpop;
  av.ll = ar->ll;
  av.gamma = ar->gamma;
  av.log_z = ar->log_z;
  av.n_used = ar->n_used;
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess)
    e = rjsmc::launch_adapt_recycled(smc_shape(c), dp, ll, gamma, log_z, n_sound, av, *prior, factors,
                                     (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_adapt_recycled: launch");
  return RJSMC_OK;
}

static rjsmc_status grad_buffer(const rjsmc_ctx *c, const rjsmc_particles *g, const rjsmc_particles *like,
                                const char *who, rjsmc::DevParticles *dp, rjsmc::DevGrad *dg) {
  rjsmc_particles tmp = *g;
  tmp.n = like->n;
  tmp.n_per_sounding = like->n_per_sounding;
  tmp.layout = like->layout;
  tmp.kappa = like->kappa;
  tmp.lambda = like->lambda;
  rjsmc_status st = check_particles(c, &tmp, who, dp);
  if (st != RJSMC_OK) return st;
  if (g->stride != like->stride) return fail(RJSMC_E_INVALID, "%s: gradient stride differs from the state's", who);
  *dg = rjsmc::DevGrad{g->phi_b, g->phi, g->z_cond, g->m, g->z_charg, g->log10_tau, g->c};
  return RJSMC_OK;
}

// The sweeps of rjsmc_mutate with the per-particle scratch `ws` (the context's workspace
// or the static scratch); allocates nothing.
static rjsmc_status mutate_impl(const char *who, rjsmc_ctx *c, const rjsmc_mutate_args *a, rjsmc_particles *state,
                                double *ll, rjsmc_particles *scratch, double *ll_scratch, const double *gamma,
                                const int32_t *active, const double *y_obs, rjsmc_particles *grad_cur,
                                rjsmc_particles *grad_prop, int64_t *stats, rjsmc_stream stream,
                                const rjsmc::MutateWorkspace &ws, const char *ws_name) {
  rjsmc::DevParticles ds, dq;
  rjsmc_status st = check_particles(c, state, who, &ds);
  if (st == RJSMC_OK) st = check_particles(c, scratch, who, &dq);
  if (st != RJSMC_OK) return st;
  if (state->layout != RJSMC_LAYOUT_DECOUPLED || scratch->layout != RJSMC_LAYOUT_DECOUPLED)
    return fail(RJSMC_E_INVALID, "%s: DECOUPLED layout only", who);
  if (scratch->n != state->n || scratch->n_per_sounding != state->n_per_sounding)
    return fail(RJSMC_E_INVALID, "%s: scratch and state differ in shape", who);
  if (state->n > ws.n || !ws.mask)
    return fail(RJSMC_E_INVALID, "%s: n=%lld exceeds %s=%lld", who, (long long)state->n, ws_name, (long long)ws.n);
  if (!ll || !ll_scratch || !gamma || !y_obs) return fail(RJSMC_E_INVALID, "%s: NULL array", who);
  if ((st = check_prior(&a->prior, who)) != RJSMC_OK) return st;
  if ((st = check_soundings(state, a->n_sound, who)) != RJSMC_OK) return st;
  if (a->n_moves < 0) return fail(RJSMC_E_INVALID, "%s: negative n_moves", who);
  double total = 0;
  for (int t = 0; t < RJSMC_N_MOVES; ++t) {
    if (!(a->move_prob[t] >= 0)) return fail(RJSMC_E_INVALID, "%s: negative move probability", who);
    total += a->move_prob[t];
  }
  if (!(total > 0)) return fail(RJSMC_E_INVALID, "%s: move probabilities sum to zero", who);
  const bool mala = a->move_prob[RJSMC_MOVE_WITHIN_MALA] > 0;
  if ((a->move_prob[RJSMC_MOVE_WITHIN_RW] > 0 || mala) && !a->factors)
    return fail(RJSMC_E_INVALID, "%s: within-model moves need proposal factors", who);
  if (a->zca_birth != 0 && a->zca_birth != 1) return fail(RJSMC_E_INVALID, "%s: zca_birth must be 0 or 1", who);
  if (a->zca_birth && !a->factors) return fail(RJSMC_E_INVALID, "%s: adaptive births need proposal factors", who);
  if (!(a->z_move_sd >= 0) || !(a->rw_scale >= 0) || !(a->mala_eps >= 0))
    return fail(RJSMC_E_INVALID, "%s: bad step sizes", who);
  rjsmc::DevParticles gcd, gpd;
  rjsmc::DevGrad gcw, gpw;
  if (mala) {
    if (c->precision != RJSMC_F64)
      return fail(RJSMC_E_UNSUPPORTED, "%s: gradient-informed moves need an FP64 context", who);
    if (!grad_cur || !grad_prop) return fail(RJSMC_E_INVALID, "%s: gradient-informed moves need gradient buffers", who);
    if ((st = grad_buffer(c, grad_cur, state, who, &gcd, &gcw)) != RJSMC_OK) return st;
    if ((st = grad_buffer(c, grad_prop, scratch, who, &gpd, &gpw)) != RJSMC_OK) return st;
  }
  const rjsmc::SmcShape sh = smc_shape(c);
  hipError_t e = hipSetDevice(c->device);
  hipStream_t s = (hipStream_t)stream;
  rjsmc::DevParticles prop1 = dq, prop2 = dq, cur2 = ds;
  prop1.mask = ws.mask;
  prop1.mask_value = 1;
  prop2.mask = ws.mask;
  prop2.mask_value = 2;
  cur2.mask = ws.mask;
  cur2.mask_value = 2;
  if (a->trial < 0 || a->trial > 1000) return fail(RJSMC_E_INVALID, "%s: trial=%d outside 0..1000", who, a->trial);
  // Langevin moves keep each particle's current gradient from sweep to sweep until an
  // accepted move of another type changes the state
  int32_t *gvalid = mala ? ws.gvalid : nullptr;
  rjsmc::DevParticlesW gcw_state = mala ? writable(gcd) : rjsmc::DevParticlesW();
  if (a->keep_gradients != 0 && a->keep_gradients != 1)
    return fail(RJSMC_E_INVALID, "%s: keep_gradients must be 0 or 1", who);
  if (e == hipSuccess && gvalid && !a->keep_gradients) e = rjsmc::launch_fill_i32(gvalid, ds.n, 0, s);
  // without gradient moves, the decision of a sweep and the proposal of the next share a
  // launch (both per particle)
  const bool fuse = !mala;
  for (int r0 = 0; r0 < a->n_moves && e == hipSuccess; ++r0) {
    const int r = a->trial * (1 << 20) + r0;   // random-number move index
    if (fuse) {
      if (r0 == 0)
        e = rjsmc::launch_propose(sh, *a, r, ds, writable(dq), ws.mask, ws.type, gamma, nullptr, nullptr, ws.lq,
                                  active, true, s);
      else
        e = rjsmc::launch_accept_propose(sh, *a, r - 1, r, writable(ds), ll, writable(dq), ll_scratch, ws.mask,
                                         ws.type, gamma, stats, ws.lq, active, s);
      if (e == hipSuccess) e = run_forward(c, prop1, c->tuning, nullptr, y_obs, ll_scratch, s, &ws);
      if (e == hipSuccess && r0 + 1 == a->n_moves)
        e = rjsmc::launch_accept(sh, *a, r, writable(ds), ll, dq, ll_scratch, ws.mask, ws.type, gamma, nullptr,
                                 nullptr, nullptr, stats, ws.lq, s);
      continue;
    }
    if (mala) {
      e = rjsmc::launch_draw_types(*a, r, ds, sh.kc, sh.km, ws.mask, ws.type, active, gvalid, s);
      if (e == hipSuccess)   // gradients of the current states of the particles taking a Langevin step
        e = rjsmc::launch_loglik_grad(c->dev, cur2, c->kmax_cond, c->kmax_charg, y_obs, ll_scratch, gcw, s, &ws);
    }
    if (e == hipSuccess)   // without gradient moves the proposal kernel draws the types itself
      e = rjsmc::launch_propose(sh, *a, r, ds, writable(dq), ws.mask, ws.type, gamma, mala ? &gcd : nullptr,
                                gvalid, ws.lq, active, !mala, s);
    if (e == hipSuccess)
      e = run_forward(c, prop1, c->tuning, nullptr, y_obs, ll_scratch, s, &ws);
    if (e == hipSuccess && mala)
      e = rjsmc::launch_loglik_grad(c->dev, prop2, c->kmax_cond, c->kmax_charg, y_obs, ll_scratch, gpw, s, &ws);
    if (e == hipSuccess)
      e = rjsmc::launch_accept(sh, *a, r, writable(ds), ll, dq, ll_scratch, ws.mask, ws.type, gamma,
                               mala ? &gcw_state : nullptr, mala ? &gpd : nullptr, gvalid, stats, ws.lq, s);
  }
  if (e != hipSuccess) {
    char what[96];
    snprintf(what, sizeof what, "%s: launch", who);
    return hip_fail(e, what);
  }
  return RJSMC_OK;
}

extern "C" rjsmc_status rjsmc_mutate(rjsmc_ctx *c, const rjsmc_mutate_args *a, rjsmc_particles *state, double *ll,
                                     rjsmc_particles *scratch, double *ll_scratch, const double *gamma,
                                     const int32_t *active, const double *y_obs, rjsmc_particles *grad_cur,
                                     rjsmc_particles *grad_prop, int64_t *stats, rjsmc_stream stream) {
  const char *who = "rjsmc_mutate";
  if (!c || !a) return fail(RJSMC_E_INVALID, "%s: NULL argument", who);
  const rjsmc::MutateWorkspace ws = ctx_workspace(c);
  return mutate_impl(who, c, a, state, ll, scratch, ll_scratch, gamma, active, y_obs, grad_cur, grad_prop, stats,
                     stream, ws, "the context's max_particles");
}

extern "C" rjsmc_status rjsmc_mutate_noalloc(rjsmc_ctx *c, const rjsmc_mutate_args *a, rjsmc_particles *state,
                                             double *ll, rjsmc_particles *scratch, double *ll_scratch,
                                             const double *gamma, const int32_t *active, const double *y_obs,
                                             rjsmc_particles *grad_cur, rjsmc_particles *grad_prop, int64_t *stats,
                                             rjsmc_stream stream) {
  const char *who = "rjsmc_mutate_noalloc";
  if (!c || !a) return fail(RJSMC_E_INVALID, "%s: NULL argument", who);
  rjsmc::MutateWorkspace ws;
  if (!rjsmc::static_scratch(c->device, &ws))
    return fail(RJSMC_E_DEVICE, "%s: the static scratch of device %d is unavailable: %s", who, c->device,
                hipGetErrorString(rjsmc::static_scratch_status(c->device)));
  return mutate_impl(who, c, a, state, ll, scratch, ll_scratch, gamma, active, y_obs, grad_cur, grad_prop, stats,
                     stream, ws, "RJSMC_NOALLOC_MAX_PARTICLES");
}

// ---------------------------------------------------------------------------- tuning
// (waves_per_block, waves_per_particle) of the compiled tile shapes.
static const int kShapes[RJSMC_TUNING_CANDIDATES / 2][2] = {{2, 1}, {4, 1}, {8, 1}, {2, 2},
                                                            {1, 4}, {1, 8}, {1, 16}, {16, 0}};

static bool valid_tuning(const rjsmc_tuning &t) {
  if (t.layer_sort != 0 && t.layer_sort != 1) return false;
  for (const auto &sh : kShapes)
    if (t.waves_per_block == sh[0] && t.waves_per_particle == sh[1]) return true;
  return false;
}

// Whether a workgroup of the tile shape fits the device's LDS for this system: the
// shapes that split the filter abscissae among waves stage every reflection term in
// LDS, which long filters and many frequencies can push beyond the limit.
static bool tuning_fits(const rjsmc_ctx *c, const rjsmc_tuning &t, size_t *need) {
  size_t bytes = 0;
  if (rjsmc::forward_lds_bytes(c->dev, c->precision, t.waves_per_block, t.waves_per_particle, &bytes) != hipSuccess)
    return false;
  if (need) *need = bytes;
  return bytes <= c->lds_limit;
}

extern "C" rjsmc_status rjsmc_set_tuning(rjsmc_ctx *c, const rjsmc_tuning *t) {
  if (!c || !t) return fail(RJSMC_E_INVALID, "rjsmc_set_tuning: NULL argument");
  if (!valid_tuning(*t))
    return fail(RJSMC_E_INVALID, "rjsmc_set_tuning: (%d, %d, %d) is not a compiled tile shape", t->waves_per_block,
                t->layer_sort, t->waves_per_particle);
  if (t->waves_per_particle == 0 && c->precision != RJSMC_F64)
    return fail(RJSMC_E_INVALID, "rjsmc_set_tuning: the spread evaluation (%d, %d, 0) runs in FP64 contexts only",
                t->waves_per_block, t->layer_sort);
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_set_tuning: hipSetDevice");
  size_t need = 0;
  if (!tuning_fits(c, *t, &need))
    return fail(RJSMC_E_INVALID, "rjsmc_set_tuning: (%d, %d, %d) needs %zu bytes of LDS per workgroup, more than %zu",
                t->waves_per_block, t->layer_sort, t->waves_per_particle, need, c->lds_limit);
  c->tuning = *t;
  return RJSMC_OK;
}

extern "C" rjsmc_status rjsmc_get_tuning(const rjsmc_ctx *c, rjsmc_tuning *t) {
  if (!c || !t) return fail(RJSMC_E_INVALID, "rjsmc_get_tuning: NULL argument");
  *t = c->tuning;
  return RJSMC_OK;
}

extern "C" rjsmc_status rjsmc_autotune(rjsmc_ctx *c, const rjsmc_particles *p, const double *y_obs, double *ll,
                                       int32_t reps, rjsmc_tuning *best, float *times_ms, rjsmc_stream stream) {
  const char *who = "rjsmc_autotune";
  if (!c) return fail(RJSMC_E_INVALID, "%s: NULL context", who);
  rjsmc::DevParticles dp;
  rjsmc_status st = check_particles(c, p, who, &dp);
  if (st != RJSMC_OK) return st;
  if (!y_obs || !ll) return fail(RJSMC_E_INVALID, "%s: NULL y_obs or ll", who);
  if (reps < 1 || reps > 1000) return fail(RJSMC_E_INVALID, "%s: reps=%d outside 1..1000", who, reps);
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_autotune: hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  e = hipEventCreate(&ev0);
  if (e == hipSuccess) e = hipEventCreate(&ev1);
  rjsmc_tuning bt = c->tuning;
  float bms = -1.0f;
  for (int k = 0; k < RJSMC_TUNING_CANDIDATES && e == hipSuccess; ++k) {
    const rjsmc_tuning t = {kShapes[k / 2][0], k % 2, kShapes[k / 2][1]};
    float ms = -1.0f;
    const bool spread = t.waves_per_particle == 0;
    const bool spread_ok = c->precision == RJSMC_F64 && c->work_rim && dp.n <= c->work_rim_n;
    if ((!t.layer_sort || (c->work_perm && dp.n <= c->work_n)) && (!spread || spread_ok) &&
        tuning_fits(c, t, nullptr)) {
      e = run_forward(c, dp, t, nullptr, y_obs, ll, s);   // warm-up
      if (e == hipSuccess) e = hipEventRecord(ev0, s);
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = run_forward(c, dp, t, nullptr, y_obs, ll, s);
      if (e == hipSuccess) e = hipEventRecord(ev1, s);
      if (e == hipSuccess) e = hipEventSynchronize(ev1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
      if (e == hipSuccess) {
        ms /= (float)reps;
        if (bms < 0 || ms < bms) {
          bms = ms;
          bt = t;
        }
      }
    }
    if (times_ms) times_ms[k] = ms;
  }
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_autotune");
  c->tuning = bt;
  if (best) *best = bt;
  return RJSMC_OK;
}

extern "C" rjsmc_status rjsmc_counter_add(rjsmc_ctx *c, int32_t *counter, int32_t delta, rjsmc_stream stream) {
  if (!c || !counter) return fail(RJSMC_E_INVALID, "rjsmc_counter_add: NULL argument");
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = rjsmc::launch_counter_add(counter, delta, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_counter_add: launch");
  return RJSMC_OK;
}

extern "C" rjsmc_status rjsmc_summarize(rjsmc_ctx *c, const rjsmc_particles *p, const rjsmc_summary_args *a,
                                        rjsmc_stream stream) {
  const char *who = "rjsmc_summarize";
  if (!c || !a) return fail(RJSMC_E_INVALID, "%s: NULL argument", who);
  rjsmc::DevParticles dp;
  rjsmc_status st = check_particles(c, p, who, &dp);
  if (st != RJSMC_OK) return st;
  if ((st = check_soundings(p, a->n_sound, who)) != RJSMC_OK) return st;
  if (a->n_depth < 0 || a->n_depth > 65536) return fail(RJSMC_E_INVALID, "%s: n_depth=%d outside 0..65536", who, a->n_depth);
  if (a->n_depth > 0 && !a->depth_m) return fail(RJSMC_E_INVALID, "%s: NULL depth grid", who);
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = rjsmc::launch_summary(smc_shape(c), dp, *a, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_summarize: launch");
  return RJSMC_OK;
}

extern "C" rjsmc_status rjsmc_posterior_predictive(rjsmc_ctx *c, const rjsmc_particles *p, const rjsmc_ppd_args *a,
                                                   rjsmc_stream stream) {
  const char *who = "rjsmc_posterior_predictive";
  if (!c || !a) return fail(RJSMC_E_INVALID, "%s: NULL argument", who);
  rjsmc::DevParticles dp;
  rjsmc_status st = check_particles(c, p, who, &dp);
  if (st != RJSMC_OK) return st;
  const int64_t nps = p->n_per_sounding > 0 ? p->n_per_sounding : p->n;
  if (a->n_sound < 1 || nps * (int64_t)a->n_sound != p->n)
    return fail(RJSMC_E_INVALID, "%s: n_sound=%d does not tile n=%lld", who, a->n_sound, (long long)p->n);
  if (!a->y_obs || !a->resp || !a->mean || !a->sd) return fail(RJSMC_E_INVALID, "%s: NULL array", who);
  hipError_t e = hipSetDevice(c->device);
  hipStream_t s = (hipStream_t)stream;
  if (e == hipSuccess) e = run_forward(c, dp, c->tuning, a->resp, nullptr, nullptr, s);
  if (e == hipSuccess) e = rjsmc::launch_ppd(c->dev, dp, a->n_sound, a->resp, a->y_obs, a->mean, a->sd, a->z, s);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_posterior_predictive: launch");
  return RJSMC_OK;
}

extern "C" rjsmc_status rjsmc_scale_bisect(rjsmc_ctx *c, const rjsmc_bisect_args *a, rjsmc_stream stream) {
  const char *who = "rjsmc_scale_bisect";
  if (!c || !a) return fail(RJSMC_E_INVALID, "%s: NULL argument", who);
  if (a->n_sound < 1) return fail(RJSMC_E_INVALID, "%s: n_sound < 1", who);
  if (!a->log_lo || !a->log_hi || !a->scale || !a->stats_sound) return fail(RJSMC_E_INVALID, "%s: NULL array", who);
  if (a->init && !(a->lo0 > 0 && a->hi0 > a->lo0 && std::isfinite(a->hi0)))
    return fail(RJSMC_E_INVALID, "%s: bad initial bracket", who);
  if (!(a->target > 0 && a->target < 1)) return fail(RJSMC_E_INVALID, "%s: target outside (0, 1)", who);
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = rjsmc::launch_scale_bisect(*a, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_scale_bisect: launch");
  return RJSMC_OK;
}
