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
  void *ptrs[] = {d.omega, d.lam, d.ck, d.K, d.eps_an2, d.flags};
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
             {&d.eps_an2, eps2.data(), (size_t)ng}};
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
  if (e != hipSuccess) {
    free_dev(d);
    delete[] c->K_host;
    delete c;
    return hip_fail(e, "rjsmc_create: flag word");
  }
  *out = c;
  return RJSMC_OK;
}

extern "C" void rjsmc_destroy(rjsmc_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
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
  return RJSMC_OK;
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
    e = rjsmc::launch_forward(c->dev, dp, c->kmax_cond, c->kmax_charg, c->precision, resp, nullptr,
                              nullptr, (hipStream_t)stream);
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
    e = rjsmc::launch_forward(c->dev, dp, c->kmax_cond, c->kmax_charg, c->precision, nullptr, y_obs,
                              ll, (hipStream_t)stream);
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
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess)
    e = rjsmc::launch_loglik_grad(c->dev, dp, c->kmax_cond, c->kmax_charg, y_obs, ll, g,
                                  (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rjsmc_loglik_grad: launch");
  return RJSMC_OK;
}
