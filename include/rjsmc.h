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

/* Particle layouts (paper, Section 2.1 and Fig. 2).
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
  int64_t max_particles;       /* workspace size of rjsmc_mutate (0: no mutation) */
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

/* Log-likelihood of Section 2.3.2 and its gradient with respect to every continuous
 * parameter of the particle vector of Section 2.3.1 (phi_b, phi, z_cond, m, z_charg,
 * log10_tau, c): the local derivative information of the gradient-informed within-model
 * proposals that Section 3 cites (Langevin, Riemann-manifold samplers).  By a reverse sweep through
 * the log-likelihood, time transform, Hankel filter, reflection recursion, Cole-Cole
 * terms and the merge.  `grad` has the particle layout and shapes (its count and
 * layout fields are ignored); slots outside each particle's counts are written 0.
 * FP64 only (RJSMC_E_UNSUPPORTED for an FP32 context). */
rjsmc_status rjsmc_loglik_grad(rjsmc_ctx *ctx, const rjsmc_particles *p, const double *y_obs,
                               double *ll, rjsmc_particles *grad, rjsmc_stream stream);

/* ------------------------------------------------------------------------------------
 * SMC primitives (Algorithm 1).  All arithmetic on weights, temperatures and evidence
 * is FP64.  Particles of one sounding are contiguous; n_sound soundings of
 * n_per_sounding particles each (n_per_sounding = 0: one sounding of n).  Model index
 * k = kappa (kmax_charg + 1) + lambda; n_models = (kmax_cond + 1)(kmax_charg + 1).
 * Random numbers: Philox4x32-10 keyed by `seed`; particle i at step t, move r uses
 * counters (i, t, r, slot); resampling of model k of sounding s uses (s, t, k, 2^31);
 * prior draws use (i, 0, slot, 2^30).  Uniforms are (x + 0.5) 2^-53 for 53-bit x.
 * ---------------------------------------------------------------------------------- */

/* Particles per sounding that the SMC calls accept (the paper's field inversions used
 * 9,600; Section 4.2). */
#define RJSMC_MAX_PER_SOUNDING 10240

/* Bounds of the uniform priors (Section 2.3.1); depths are uniform on (0, z_max) of
 * the context and the counts are uniform on 0..kmax of the context. */
typedef struct {
  double phi_lo, phi_hi;        /* log10 sigma_inf */
  double m_lo, m_hi;            /* chargeability */
  double ltau_lo, ltau_hi;      /* log10 tau */
  double c_lo, c_hi;            /* Cole-Cole exponent */
} rjsmc_prior;

/* Draws every particle of `p` (DECOUPLED layout, device memory, counts and values
 * written) from the prior (Algorithm 1 initialisation): kappa, lambda uniform on
 * 0..kmax, properties uniform, depths sorted uniforms on (0, z_max). */
rjsmc_status rjsmc_init_prior(rjsmc_ctx *ctx, rjsmc_particles *p, const rjsmc_prior *prior,
                              uint64_t seed, rjsmc_stream stream);

typedef struct {
  double alpha_tess;            /* target fraction of the total effective sample size */
  uint64_t seed;
  int32_t step;                 /* t >= 1 */
  int32_t n_sound;
  const int32_t *step_dev;      /* device, may be NULL: when set, t is read from *step_dev
                                   when the kernels run (for replayed HIP graphs) */
} rjsmc_reweight_args;

/* Re-weight and re-sample every sounding (Algorithm 1; Section 3.2.1; Appendices C, D):
 *  - the temperature increment dg is 1 - gamma if the total effective sample size
 *    TESS(dg) = sum_k (sum_{i in k} w_i)^2 / sum_{i in k} w_i^2, w_i = exp(dg ll_i), stays
 *    >= alpha N; otherwise 60 bisection steps on (0, 1 - gamma] keep the lower bracket
 *    (TESS does not increase with dg, so the kernel evaluates it only at the midpoints
 *    inside a bracket it first narrows by Newton steps; the other decisions follow from
 *    the bracket ends).  A particle with ll = -inf has weight 0, also when dg = 0;
 *  - log_z[s][k] += logsumexp_{i in k}(dg ll_i) - ln N_k for every populated model;
 *    a model with no member has an empty sum of incremental weights, so its estimate
 *    (a product over steps) is 0 from then on: log_z[s][k] = -inf;
 *  - within each model, systematic resampling of its N_k members from the normalised
 *    weights quantised to round(W_i 2^60); member j (by particle index) receives the
 *    first member whose cumulative weight exceeds floor((j 2^53 + U) T / (N_k 2^53));
 *  - out / ll_out receive the resampled population (out may not alias in).
 * Soundings with gamma >= 1 are copied unchanged.  active[s] (device, may be NULL) is
 * set to 1 if the sounding was re-weighted, else 0.  ancestors[n] (device) receives the
 * global index of each particle's ancestor.  Requires n_per_sounding <=
 * RJSMC_MAX_PER_SOUNDING and n_models <= 128 (RJSMC_E_UNSUPPORTED otherwise). */
rjsmc_status rjsmc_reweight_resample(rjsmc_ctx *ctx, const rjsmc_reweight_args *args,
                                     const rjsmc_particles *in, const double *ll_in,
                                     rjsmc_particles *out, double *ll_out, double *gamma,
                                     double *log_z, int32_t *active, int32_t *ancestors,
                                     rjsmc_stream stream);

/* Proposal factors of the within-model move (Section 3.2.2).  For every (sounding,
 * model) with more members than dimensions d = 3 + 2 kappa + 2 lambda:
 * F = U diag(sqrt(Lambda)) from the eigen-decomposition of the members' sample
 * covariance of theta = (phi_b, phi_1..kappa, z_1..kappa, m_1..lambda, zm_1..lambda,
 * log10 tau, c); otherwise F = 0.1 diag(prior standard deviations).
 * factors: device [n_sound][n_models][dmax][dmax], column r (direction r) contiguous:
 * F[r][a] at offset r dmax + a; dmax = 3 + 2 kmax_cond + 2 kmax_charg. */
rjsmc_status rjsmc_adapt(rjsmc_ctx *ctx, const rjsmc_particles *p, int32_t n_sound,
                         const rjsmc_prior *prior, double *factors, rjsmc_stream stream);

/* Archive of earlier populations for particle recycling (Section 3.2.4).  Slot h holds
 * the population of an earlier step, in the layout of the current one (n = n_sound
 * n_per_sounding particles, soundings contiguous):
 *   particle i of slot h is column h n + i of `pop` (pop.n = n_slots n, pop.stride >=
 *   pop.n; its n_per_sounding is ignored), its log-likelihood ll[h n + i];
 *   gamma[h n_sound + s] is the temperature that slot's population targets and
 *   log_z[(h n_sound + s) n_models + k] the evidence estimate log Z_{h,k} of model k
 *   at that temperature.
 * Slots 0 .. n_used - 1 are read; n_used <= n_slots <= RJSMC_MAX_ARCHIVE.  All arrays
 * are device memory owned by the caller. */
#define RJSMC_MAX_ARCHIVE 64
typedef struct {
  rjsmc_particles pop;
  double *ll;
  double *gamma;
  double *log_z;
  int32_t n_slots, n_used;
} rjsmc_archive;

/* Copies population p (n particles, its ll, and the per-sounding gamma[n_sound] and
 * log_z[n_sound][n_models]) into slot `slot` of the archive (0 <= slot < n_slots).
 * RJSMC_E_INVALID on shape mismatch; does not change n_used. */
rjsmc_status rjsmc_archive_store(rjsmc_ctx *ctx, const rjsmc_particles *p, const double *ll,
                                 const double *gamma, const double *log_z, int32_t n_sound,
                                 rjsmc_archive *archive, int32_t slot, rjsmc_stream stream);

/* Proposal factors from recycled particles (Section 3.2.4 with Section 3.2.2).  For
 * each (sounding s, model k) the members of model k in the current population p (with
 * log-likelihoods ll, temperature gamma[s], evidence log_z[s][k]) and in the archive's
 * used slots are pooled and weighted by the deterministic mixture
 *   nu = L^gamma_t / sum_l N_l L^gamma_l / Z_{l,k}
 * over the sources l (slots and the current population) that hold N_l > 0 members of
 * model k and a finite log Z_{l,k} (L^0 = 1; the prior density cancels).  F is the
 * factor (as in rjsmc_adapt) of the weighted covariance sum w (theta - mu)(theta -
 * mu)^T / (1 - sum w^2), normalised weights w; 0.1 diag(prior sd) when the weights'
 * effective sample size (sum w)^2 / sum w^2 is not above d.  With an empty archive the
 * weights are equal and F is that of rjsmc_adapt (up to rounding). */
rjsmc_status rjsmc_adapt_recycled(rjsmc_ctx *ctx, const rjsmc_particles *p, const double *ll,
                                  const double *gamma, const double *log_z, int32_t n_sound,
                                  const rjsmc_archive *archive, const rjsmc_prior *prior,
                                  double *factors, rjsmc_stream stream);

/* Move types of the RJ-MCMC kernel (Appendix E.1; Section 3.2.2). */
enum {
  RJSMC_MOVE_SIGMA_BIRTH = 0, RJSMC_MOVE_SIGMA_DEATH = 1, RJSMC_MOVE_SIGMA_MOVE = 2,
  RJSMC_MOVE_M_BIRTH = 3, RJSMC_MOVE_M_DEATH = 4, RJSMC_MOVE_M_MOVE = 5,
  RJSMC_MOVE_WITHIN_RW = 6, RJSMC_MOVE_WITHIN_MALA = 7, RJSMC_N_MOVES = 8
};

typedef struct {
  uint64_t seed;
  int32_t step;                 /* t */
  int32_t n_moves;              /* R: sweeps of every particle */
  int32_t n_sound;
  double move_prob[8];          /* relative probability of each move type */
  double z_move_sd;             /* sd of an interface move (m) */
  double rw_scale;              /* within-model step along a principal direction */
  double mala_eps;              /* gradient-informed step size */
  const double *factors;        /* device, as written by rjsmc_adapt */
  rjsmc_prior prior;
  const int32_t *step_dev;      /* device, may be NULL: when set, t is read from *step_dev */
  const double *rw_scale_dev;   /* device [n_sound], may be NULL: per-sounding within-model
                                   step (overrides rw_scale) */
  int64_t *stats_sound;         /* device [n_sound][2], may be NULL: within-model (random-walk
                                   or gradient-informed) proposals / acceptances per sounding
                                   (accumulated) */
  int32_t trial;                /* 0: the sweeps of Algorithm 1.  b >= 1: trial proposals
                                   (Section 3.2.2) decided and counted but never kept, with
                                   random-number move index b * 2^20 + r */
  int32_t zca_birth;            /* 0: a birth draws the new property from its prior.  1: the
                                   adaptive birth and death of Appendix E.2: the new depth
                                   u_d = z_max u fixes the insertion index r, the split
                                   segment's property (0 above the first chargeability
                                   interface) is copied below the new interface, and every
                                   other component of the larger model's vector is shifted
                                   by S[i, :] u_p, u_p ~ N(0, 1), with S = sum_r f_r f_r^T /
                                   |f_r| the symmetric root of the larger model's F F^T
                                   (from `factors`) and i the new property's component;
                                   the MH ratio gains log|S[i, new] - S[i, source]| -
                                   log(prior range) - log phi(u_p) (its negative for the
                                   death, which inverts the map with the same S and is
                                   rejected unless the recovered state is in the support
                                   with u_d at index r) */
  const double *mala_eps_dev;   /* device [n_sound], may be NULL: per-sounding step of the
                                   gradient-informed move (overrides mala_eps), e.g. bisected
                                   from trial proposals toward a target acceptance as the
                                   random-walk scale is (Section 3.2.2) */
  int32_t keep_gradients;       /* 0: the gradients of the current states are recomputed when
                                   a gradient-informed move needs them (validity cleared at the
                                   call's start).  1: the gradients in grad_cur, and which of
                                   them are valid, carry over from the previous rjsmc_mutate
                                   call on this context; the caller guarantees that neither the
                                   states nor grad_cur changed in between (e.g. successive trial
                                   calls, which never change the states, and the call after
                                   them) */
} rjsmc_mutate_args;

/* n_moves RJ-MCMC sweeps (Algorithm 1, mutation) targeting L^gamma(sounding) x prior.
 * Per sweep every particle of an active sounding proposes one move of a type drawn from
 * move_prob: birth (depth uniform on (0, z_max), property from its prior), death (a
 * uniformly chosen interface), move (one depth + N(0, z_move_sd^2)), a within-model step
 * theta + rw_scale xi F[:, r] along a uniformly chosen principal direction r, or a
 * gradient-informed (preconditioned Langevin) step
 *   theta' = theta + mala_eps^2/2 F F^T gamma grad ll + mala_eps F xi
 * whose acceptance includes the reverse-proposal correction
 *   -|xi + mala_eps/2 F^T gamma (grad ll + grad' ll)|^2 / 2 + |xi|^2 / 2.
 * Proposals beyond the capacities or outside the prior support are rejected; the others
 * are accepted when ln u < gamma (ll' - ll) (+ the correction).  `scratch` and
 * `ll_scratch` hold the proposals (same shapes as `state`).  grad_cur and grad_prop
 * (device, particle-shaped, may be NULL unless move_prob[WITHIN_MALA] > 0) receive
 * gradients of the current states and of the proposals; gradient-informed moves need an
 * FP64 context.  n must not exceed the context's max_particles.  stats (device int64
 * [2][8], may be NULL) accumulates proposed / accepted counts per move type.  active
 * (device [n_sound], NULL = all) selects soundings. */
rjsmc_status rjsmc_mutate(rjsmc_ctx *ctx, const rjsmc_mutate_args *args, rjsmc_particles *state,
                          double *ll, rjsmc_particles *scratch, double *ll_scratch,
                          const double *gamma, const int32_t *active, const double *y_obs,
                          rjsmc_particles *grad_cur, rjsmc_particles *grad_prop, int64_t *stats,
                          rjsmc_stream stream);

/* Allocation-free variant of rjsmc_mutate, for callers that cannot allocate device
 * memory at the time of the call: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, behaviour and results as
 * rjsmc_mutate (bit-identical), except that the per-particle scratch of the sweeps
 * (proposal mask, move type, gradient validity, adaptive-birth correction, evaluation
 * order) lives in a static device array of the library instead of the context's
 * workspace, so the context may have been created with max_particles = 0.  That array
 * holds RJSMC_NOALLOC_MAX_PARTICLES particles (about 6 MiB per GPU, kept until the
 * process ends); a larger state->n gives RJSMC_E_INVALID before anything is enqueued.
 * Every call on one GPU uses that GPU's one array: calls that overlap on a GPU (other
 * streams, other threads, other contexts) race and must be serialised by the caller.
 * The call allocates nothing, also not on the host side of the runtime. */
#define RJSMC_NOALLOC_MAX_PARTICLES 262144
rjsmc_status rjsmc_mutate_noalloc(rjsmc_ctx *ctx, const rjsmc_mutate_args *args, rjsmc_particles *state,
                                  double *ll, rjsmc_particles *scratch, double *ll_scratch,
                                  const double *gamma, const int32_t *active, const double *y_obs,
                                  rjsmc_particles *grad_cur, rjsmc_particles *grad_prop, int64_t *stats,
                                  rjsmc_stream stream);

/* Posterior summaries of a population (Section 2.3.3 and the case studies), per sounding:
 *  - model_count[s][k]: particles in model k (pi_T(k | y) = count / N, Section 3.2.1);
 *  - log_bfipd[s]: log of the grouped Bayes factor of chargeable (lambda >= 1) versus
 *    conductive-only (lambda = 0) models with the uniform model prior,
 *      log[(n_charg / |M_charg|) / (n_cond / |M_cond|)]
 *        = log n_charg - log n_cond - log kmax_charg,
 *    +inf when no particle is conductive-only, -inf when none is chargeable, NaN for the
 *    MERGED layout or kmax_charg = 0;
 *  - at each depth z of depth_m: the model-averaged mean of log10 sigma_inf(z) and of
 *    m(z), and the fraction of particles with m(z) > 0 (a property applies from its
 *    interface down, as in the merge).
 * Output pointers are device memory and may be NULL (that output is skipped).
 * Sums run over the particles in index order (reproducible). */
typedef struct {
  int32_t n_sound;
  int32_t n_depth;              /* 0 .. 65536 */
  const double *depth_m;        /* device [n_depth] */
  int32_t *model_count;         /* device [n_sound][n_models] */
  double *log_bfipd;            /* device [n_sound] */
  double *mean_log10_sigma;     /* device [n_sound][n_depth] */
  double *mean_m;               /* device [n_sound][n_depth] */
  double *p_chargeable;         /* device [n_sound][n_depth] */
} rjsmc_summary_args;

rjsmc_status rjsmc_summarize(rjsmc_ctx *ctx, const rjsmc_particles *p, const rjsmc_summary_args *args,
                             rjsmc_stream stream);

/* Posterior predictive summaries of each sounding's population (Section 4.1: posterior
 * predictive checks; Section 4.2: the data standardised to the posterior predictive
 * distribution at each gate).  Replicated data are y~ = y(theta) + e, e ~ N(0, Sigma(y)) with
 * the noise model of Section 2.3.2 and theta drawn from the population (equal weights, as
 * after the last mutation of Algorithm 1).  Per sounding s and gate g:
 *   mean[s][g] = (1/N) sum_i y_ig,
 *   sd[s][g]   = sqrt((1/N) sum_i (y_ig - mean)^2 + (1/N) sum_i (eps_an_g^2 + (eps_mn y_ig)^2))
 *                (law of total variance),
 *   z[s][g]    = (y_obs[s][g] - mean[s][g]) / sd[s][g]   (|z| <= 1 within one sd).
 * The forward responses of every particle are written to resp first (the forward model
 * with the context's tile shape); sums run over the sounding's particles in index order.
 * A particle with an invalid stack has NaN responses, which make its sounding's
 * summaries NaN.  All pointers are device memory; z may be NULL. */
typedef struct {
  int32_t n_sound;
  const double *y_obs;          /* [n_sound][n_gate] */
  double *resp;                 /* [n][n_gate], receives the particles' responses */
  double *mean, *sd, *z;        /* [n_sound][n_gate] */
} rjsmc_ppd_args;

rjsmc_status rjsmc_posterior_predictive(rjsmc_ctx *ctx, const rjsmc_particles *p, const rjsmc_ppd_args *args,
                                        rjsmc_stream stream);

/* One bisection step per sounding on log(scale) of the within-model random walk, from
 * trial proposals at the bracket's midpoint (Section 3.2.2: the step is scaled to reach a
 * target acceptance rate).  init = 1 starts the bracket [log lo0, log hi0]; otherwise a
 * sounding whose trials were accepted at a rate above `target` raises the lower end to
 * the midpoint, else lowers the upper end (no trials: unchanged).  Then scale =
 * exp(midpoint) and stats_sound is zeroed for the next trials.  Device arrays; no host
 * synchronisation, so it can sit inside a captured step. */
typedef struct {
  int32_t n_sound;
  int32_t init;
  double target;
  double lo0, hi0;              /* initial bracket of the scale, 0 < lo0 < hi0 */
  double *log_lo, *log_hi;      /* device [n_sound] */
  double *scale;                /* device [n_sound] */
  int64_t *stats_sound;         /* device [n_sound][2] */
} rjsmc_bisect_args;

rjsmc_status rjsmc_scale_bisect(rjsmc_ctx *ctx, const rjsmc_bisect_args *args, rjsmc_stream stream);

/* *counter += delta on the device, in stream order (one thread).  With step_dev in the
 * argument structs above, a whole SMC step (re-weight/re-sample, adapt, mutate, this
 * increment) can be captured once into a HIP graph and replayed step after step. */
rjsmc_status rjsmc_counter_add(rjsmc_ctx *ctx, int32_t *counter, int32_t delta, rjsmc_stream stream);

/* ------------------------------------------------------------------------------------
 * Tile shape of the forward kernel.  Not part of the method: it decides how the
 * particles of a launch are packed into workgroups, never what is computed (results are
 * identical for every shape).
 * ---------------------------------------------------------------------------------- */
typedef struct {
  int32_t waves_per_block;    /* particles per workgroup (spread shape: waves per workgroup) */
  int32_t layer_sort;         /* 1: evaluate particles in descending order of layer capacity
                                 (kappa + lambda + 1), computed on the device before each
                                 launch; used only when n <= max_particles of the context */
  int32_t waves_per_particle; /* wavefronts sharing one particle's frequency groups (more
                                 than one shortens the latency of small batches); 0: spread */
} rjsmc_tuning;

/* The tile shapes, as (waves_per_block, waves_per_particle):
 *   (2,1) (4,1) (8,1) (2,2) (1,4) (1,8) (1,16) (16,0),
 * each with layer_sort 0 and 1: candidate k = 2 * shape index + layer_sort.  With more
 * waves per particle than groups of 8 frequencies, each group's filter abscissae are
 * split among the waves as well (the sums keep the same order).
 * (16,0) is the spread evaluation, for small populations whose particles differ in depth:
 * each particle's reflection terms are cut into units of 64 (8 frequencies x 8 filter
 * abscissae) weighted by its layer capacity, the units are dealt in runs of equal weight
 * to the waves of one 16-wave workgroup per compute unit, and a second launch adds the
 * stored terms in the order of the other shapes.  FP64 contexts only (rjsmc_set_tuning
 * rejects it in an FP32 context, the autotuner skips it).  It needs a context workspace
 * (max_particles > 0; 8 ceil(n_freq/8) n_hankel_pad doubles per particle are allocated for
 * min(max_particles, 2048) particles); a launch over more particles than that, or from
 * rjsmc_mutate_noalloc, takes the shape (4,1) instead. */
#define RJSMC_TUNING_CANDIDATES 16

/* Sets / reads the tile shape used by rjsmc_forward, rjsmc_loglik and the proposal
 * likelihoods of rjsmc_mutate (default {4, 0, 1}).  RJSMC_E_INVALID for a shape not in
 * the list above, or for one whose workgroup needs more LDS than the device allows
 * for this system (the shapes that split the filter abscissae among waves stage
 * 8 n_freq n_hankel bytes of reflection terms per particle). */
rjsmc_status rjsmc_set_tuning(rjsmc_ctx *ctx, const rjsmc_tuning *tuning);
rjsmc_status rjsmc_get_tuning(const rjsmc_ctx *ctx, rjsmc_tuning *tuning);

/* Autotuner: times rjsmc_loglik on population p (device, as for rjsmc_loglik; ll is
 * overwritten) for every candidate tile shape, `reps` launches each after one warm-up,
 * with HIP events on `stream`; keeps the fastest in the context and writes it to *best
 * (may be NULL).  times_ms (host float[RJSMC_TUNING_CANDIDATES], may be NULL) receives
 * the mean launch time of candidate k, or -1 for a candidate that needs more workspace
 * than max_particles or more LDS than the device allows (it is skipped, not launched).
 * Synchronizes `stream`.
 * RJSMC_E_INVALID for bad arguments or reps outside 1..1000. */
rjsmc_status rjsmc_autotune(rjsmc_ctx *ctx, const rjsmc_particles *p, const double *y_obs, double *ll,
                            int32_t reps, rjsmc_tuning *best, float *times_ms, rjsmc_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* RJSMC_H */
