/*
 * rjsmc.h -- C ABI of the MI355X (gfx950) hot path of reversible-jump static
 * sequential Monte Carlo for induced-polarisation detectability in airborne EM data
 * (Davies, Ley-Cooper, Sutton, Drovandi, "Bayesian Detectability of Induced
 * Polarisation in Airborne Electromagnetic Data using Reversible Jump Sequential
 * Monte Carlo").
 *
 * Conventions for every call
 *   - Pointers inside rjsmc_particles, and the output arrays of the hot calls, are HIP
 *     device memory owned by the caller.  Pointers inside rjsmc_system are host memory
 *     and are copied by rjsmc_create.  The context owns its device tables.
 *   - Every hot call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream): it validates its arguments on the host, enqueues kernels and returns.
 *     Arguments that the host can reject (NULL pointers, n <= 0, counts beyond the
 *     context's capacities) give RJSMC_E_INVALID before anything is enqueued; a failed
 *     launch gives RJSMC_E_DEVICE.  rjsmc_last_error() returns the message of the last
 *     failure on the calling thread.
 *   - Problems only the device can see (a particle count above capacity, unsorted
 *     depths) raise a flag in the context; rjsmc_check() synchronises the stream and
 *     reports them.  A non-finite forward result is not an error: its log-likelihood is
 *     -inf so that any Metropolis-Hastings step rejects it.
 *   - Hot calls never allocate device memory.  One context per stream; a context is
 *     not thread-safe.
 */
#ifndef RJSMC_H
#define RJSMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rjsmc_ctx rjsmc_ctx;
typedef void *rjsmc_stream; /* hipStream_t */

typedef enum {
  RJSMC_OK = 0,
  RJSMC_E_INVALID = 1,
  RJSMC_E_DEVICE = 2,
  RJSMC_E_NOMEM = 3,
  RJSMC_E_CAPACITY = 4,
  RJSMC_E_UNSUPPORTED = 5
} rjsmc_status;

/* Arithmetic of the layer recursion.  RJSMC_F32 runs the Cole-Cole terms and the
 * reflection recursion in FP32 and accumulates the Hankel sum, the time transform
 * and the log-likelihood in FP64; outputs are FP64 either way. */
typedef enum { RJSMC_F64 = 0, RJSMC_F32 = 1 } rjsmc_precision;

/* Particle layouts (paper, Section 2.2 and Fig. 2).
 * DECOUPLED: two change-point partitions -- kappa conductivity interfaces and lambda
 *   chargeability interfaces -- merged by a direct sum before the forward model.
 * MERGED: one layered model of L = kappa + 1 layers, each with its own conductivity
 *   and chargeability (used for fixed-dimension forward-model throughput). */
typedef enum { RJSMC_LAYOUT_DECOUPLED = 0, RJSMC_LAYOUT_MERGED = 1 } rjsmc_layout;

/* Acquisition system and noise model (Sections 2 and 2.3.2).  Host memory. */
typedef struct {
  double loop_radius_m;        /* central loop radius a */
  double height_m;             /* transmitter/receiver height h above the ground */
  double current_a;            /* transmitter current I (step-off) */
  int32_t n_freq;              /* frequencies of the frequency-domain solve, 2..64 */
  const double *freq_hz;       /* [n_freq], strictly increasing */
  int32_t n_hankel;            /* J1 digital-filter length, 1..256 */
  const double *hankel_b;      /* [n_hankel] abscissae b_k; lam_k = b_k / a */
  const double *hankel_w;      /* [n_hankel] weights w_k */
  int32_t n_gate;              /* off-time gates, 1..32 */
  const double *gate_open_s;   /* [n_gate] gate start times (s after the step-off) */
  const double *gate_close_s;  /* [n_gate] gate end times, > gate_open_s */
  double eps_mn;               /* multiplicative noise fraction */
  const double *eps_an;        /* [n_gate] additive noise, pT/s */
  int32_t kmax_cond;           /* capacity: conductivity interfaces per particle */
  int32_t kmax_charg;          /* capacity: chargeability interfaces per particle */
  double z_max_m;              /* prior depth bound of interfaces */
  int32_t fwd_precision;       /* rjsmc_precision */
} rjsmc_system;

/* Particle population in structure-of-arrays form, particle index fastest.  Every
 * per-row array has row stride `stride` (elements; >= n).  Slots beyond a particle's
 * counts are never read.
 *   kappa[n], lambda[n]      interface counts (lambda unused for MERGED)
 *   phi_b[n]                 log10 sigma_inf of the top segment (S/m)
 *   phi[kmax_cond][stride]   log10 sigma_inf below each conductivity interface
 *   z_cond[kmax_cond][stride]   conductivity interface depths (m), ascending, >= 0
 *   m[..][stride]            DECOUPLED: chargeability below each chargeability
 *                            interface, kmax_charg rows (the top segment has m = 0);
 *                            MERGED: per-layer chargeability, kmax_cond + 1 rows
 *   z_charg[kmax_charg][stride] chargeability interface depths (DECOUPLED only)
 *   log10_tau[n], c[n]       Cole-Cole time constant (log10 s) and exponent, shared by
 *                            all chargeable layers (Section 2.3.1)
 * Particles of one sounding are contiguous: particle i belongs to sounding
 * i / n_per_sounding (n_per_sounding = 0: every particle belongs to sounding 0). */
typedef struct {
  int64_t n;
  int64_t stride;
  int64_t n_per_sounding;
  int32_t layout;              /* rjsmc_layout */
  int32_t *kappa, *lambda;
  double *phi_b, *phi, *z_cond, *m, *z_charg, *log10_tau, *c;
} rjsmc_particles;

/* Creates a context on HIP device `device` for the system `sys` (Section 2 forward
 * model).  Builds on the host, once, the frequency-to-time matrix K [n_gate][n_freq]
 * (cosine transform of the natural cubic spline of Im H / w in ln w, constant beyond
 * both ends, averaged over each boxcar gate) and the Hankel-filter coefficients
 * c_k = (I/2) w_k lam_k exp(-2 lam_k h); uploads them.  Returns RJSMC_E_INVALID for bad
 * sizes or non-increasing frequencies, RJSMC_E_NOMEM / RJSMC_E_DEVICE on HIP failures. */
rjsmc_status rjsmc_create(const rjsmc_system *sys, int device, rjsmc_ctx **out);

/* Releases the context and its device memory.  NULL is ignored. */
void rjsmc_destroy(rjsmc_ctx *ctx);

/* Message of the last failure on this thread ("" if none).  Valid until the next call. */
const char *rjsmc_last_error(void);

/* Synchronises `stream`, then reports and clears device-side flags:
 * RJSMC_E_CAPACITY if a particle exceeded the context's layer capacity,
 * RJSMC_E_INVALID if a particle had unsorted or negative depths (its outputs are NaN). */
rjsmc_status rjsmc_check(rjsmc_ctx *ctx, rjsmc_stream stream);

/* Copies the frequency-to-time matrix K [n_gate][n_freq] (row-major, pT/s per A/m)
 * into host memory `K_out`. */
rjsmc_status rjsmc_time_kernel(const rjsmc_ctx *ctx, double *K_out);

/* Host-only: builds the frequency-to-time matrix K [n_gate][n_freq] (row-major) that
 * rjsmc_create uses, for frequencies freq_hz[n_freq] (Hz, increasing) and gates
 * [gate_open_s, gate_close_s).  Needs no device.  Same sizes and errors as rjsmc_create. */
rjsmc_status rjsmc_build_time_kernel(const double *freq_hz, int32_t n_freq, const double *gate_open_s,
                                     const double *gate_close_s, int32_t n_gate, double *K_out);

/* Forward model (Section 2): for every particle, the off-time response -dBz/dt in pT/s
 * at the loop centre, averaged over each gate.  Per particle: merge the partitions
 * (Fig. 2), Cole-Cole conductivity per layer and frequency, TE reflection recursion at
 * every filter abscissa, J1 Hankel filter sum, y = K Im H.
 *   resp: device [n][n_gate] (particle-major). */
rjsmc_status rjsmc_forward(rjsmc_ctx *ctx, const rjsmc_particles *p, double *resp,
                           rjsmc_stream stream);

/* Gaussian log-likelihood of Section 2.3.2 with the diagonal covariance
 * eps_an[g]^2 + (eps_mn y_g)^2 evaluated at the model response:
 *   ll = -1/2 sum_g [(d_g - y_g)^2 / s_g^2 + ln(2 pi s_g^2)].
 *   y_obs: device [n_sound][n_gate]; ll: device [n]. */
rjsmc_status rjsmc_loglik(rjsmc_ctx *ctx, const rjsmc_particles *p, const double *y_obs,
                          double *ll, rjsmc_stream stream);

/* Log-likelihood and its gradient with respect to every continuous parameter of each
 * particle (phi_b, phi, z_cond, m, z_charg, log10_tau, c), by a reverse sweep through
 * the log-likelihood, time transform, Hankel filter, reflection recursion, Cole-Cole
 * terms and the merge.  `grad` has the particle layout and shapes (its count and
 * layout fields are ignored); slots outside each particle's counts are written 0.
 * FP64 only (RJSMC_E_UNSUPPORTED for an FP32 context). */
rjsmc_status rjsmc_loglik_grad(rjsmc_ctx *ctx, const rjsmc_particles *p, const double *y_obs,
                               double *ll, rjsmc_particles *grad, rjsmc_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* RJSMC_H */
