// Internal declarations shared by the host runtime and the HIP kernels of librjsmc.
// Not part of the public ABI (include/rjsmc.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "rjsmc.h"

namespace rjsmc {

// Compile-time limits of the kernels.
constexpr int kMaxFreq = 64;      // frequencies
constexpr int kMaxHankel = 256;   // filter abscissae
constexpr int kMaxGate = 32;      // gates
constexpr int kMaxLayers = 16;    // merged layers per particle
constexpr int kWave = 64;

// Workgroups are dealt to the eight XCDs of the chip in turn (workgroup b runs on XCD
// b mod 8), and each XCD has its own L2.  Kernels that give neighbouring particles to
// neighbouring workgroups renumber them so that each XCD takes one contiguous range:
// the particle columns' cache lines are then fetched by one L2 instead of several.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
  const uint32_t per = nb / kXcds, rem = nb % kXcds;
  const uint32_t x = b % kXcds, j = b / kXcds;
  return x * per + (x < rem ? x : rem) + j;
}

// Orders a wave's LDS writes before later LDS reads of other lanes of the same wave
// (a compiler barrier with wave-wide release/acquire; no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// Sizes of the tables of the propagation-factor exponential (see cexp_tab).
constexpr int kPhaseN = 256;
constexpr int kExp2N = 256;

// Device flag bits raised by kernels, reported by rjsmc_check.
constexpr int kFlagCapacity = 1;
constexpr int kFlagUnsorted = 2;

// Tables of one acquisition system, resident in device memory.
struct DevSystem {
  int n_freq, n_hankel, n_hankel_pad, n_gate;
  double eps_mn;
  double *omega;      // [n_freq] angular frequency
  double *lam;        // [n_hankel_pad] filter wavenumbers b_k / a (padding: 1.0)
  double *ck;         // [n_hankel_pad] (I/2) w_k lam_k exp(-2 lam_k h)  (padding: 0)
  double *K;          // [n_gate][n_freq] frequency-to-time matrix
  double *eps_an2;    // [n_gate] eps_an^2
  double *phase;      // [kPhaseN][2] (cos, sin)(j pi/128), j = 0..255
  double *exp2t;      // [kExp2N] 2^(j/256), j = 0..255
  int *flags;         // device flag word
};

// Particle pointers and sizes as the kernels see them.
struct DevParticles {
  int64_t n = 0, stride = 0, n_per_sounding = 0;
  int layout = 0;
  const int32_t *kappa = nullptr, *lambda = nullptr;
  const double *phi_b = nullptr, *phi = nullptr, *z_cond = nullptr, *m = nullptr, *z_charg = nullptr,
               *log10_tau = nullptr, *c = nullptr;
  const int32_t *mask = nullptr;   // optional: only particles with mask[i] == mask_value are
  int mask_value = 1;              // evaluated; the others are left untouched
};

// Writable view of a particle population.
struct DevParticlesW {
  int64_t n = 0, stride = 0, n_per_sounding = 0;
  int layout = 0;
  int32_t *kappa = nullptr, *lambda = nullptr;
  double *phi_b = nullptr, *phi = nullptr, *z_cond = nullptr, *m = nullptr, *z_charg = nullptr,
         *log10_tau = nullptr, *c = nullptr;
};

struct SmcShape {
  int kc, km;          // capacities
  int n_models;        // (kc+1)(km+1)
  int dmax;            // 3 + 2 kc + 2 km
  double z_max;
};

struct DevGrad {
  double *phi_b, *phi, *z_cond, *m, *z_charg, *log10_tau, *c;
};

// Tile shape of one forward launch: particles per workgroup and an optional evaluation
// order (a permutation of the particle indices).
struct ForwardTiles {
  int waves_per_block = 4;     // particles per workgroup
  int waves_per_particle = 1;  // waves sharing one particle's frequency groups; 0: spread
  const int32_t *perm = nullptr;
  // spread evaluation (waves_per_particle 0, waves_per_block 16): one workgroup per compute
  // unit, reflection terms in rim ([rim_n] slots of spread_rim_doubles(s, 1)) and layer
  // counts in rim_layers; a launch beyond rim_n particles takes the (4, 1) shape instead
  int n_cu = 0;
  double *rim = nullptr;
  int32_t *rim_layers = nullptr;
  int64_t rim_n = 0;
};
// Doubles of reflection terms the spread evaluation stores for n particles, and the most
// particles one spread launch takes.
int64_t spread_rim_doubles(const DevSystem &s, int64_t n);
int64_t spread_max_particles();

// Kernel launchers (forward.hip / adjoint.hip).  Return the launch's hipError_t.
hipError_t launch_forward(const DevSystem &s, const DevParticles &p, int kmax_cond, int kmax_charg,
                          int precision, double *resp, const double *y_obs, double *ll,
                          hipStream_t stream, const ForwardTiles &tiles);
// Static plus dynamic LDS bytes of one forward workgroup of the given tile shape for
// system s (hipErrorInvalidValue for a shape that is not compiled).
hipError_t forward_lds_bytes(const DevSystem &s, int precision, int waves_per_block, int waves_per_particle,
                             size_t *bytes);
// perm[0..n) = particle indices in descending order of layer capacity (kappa + lambda + 1);
// cnt: 2 kMaxLayers ints of device scratch.
hipError_t launch_layer_sort(const DevParticles &p, int *cnt, int32_t *perm, hipStream_t stream);
struct MutateWorkspace;
// ws (may be NULL): an evaluation-order workspace, with which particles of a context of
// more than 8 layers' capacity are split by their own capacity between instantiations.
hipError_t launch_loglik_grad(const DevSystem &s, const DevParticles &p, int kmax_cond,
                              int kmax_charg, const double *y_obs, double *ll, const DevGrad &g,
                              hipStream_t stream, const MutateWorkspace *ws = nullptr);

// SMC launchers (smc.hip).
hipError_t launch_counter_add(int32_t *counter, int32_t delta, hipStream_t stream);
hipError_t launch_scale_bisect(const rjsmc_bisect_args &a, hipStream_t stream);
hipError_t launch_summary(const SmcShape &sh, const DevParticles &p, const rjsmc_summary_args &a, hipStream_t stream);
hipError_t launch_ppd(const DevSystem &sys, const DevParticles &p, int n_sound, const double *resp,
                      const double *y_obs, double *mean, double *sd, double *z, hipStream_t stream);
hipError_t launch_init_prior(const DevParticlesW &p, const SmcShape &sh, const rjsmc_prior &pr, uint64_t seed,
                             hipStream_t stream);
hipError_t launch_reweight_resample(const SmcShape &sh, const rjsmc_reweight_args &a, const DevParticles &in,
                                    const double *ll_in, const DevParticlesW &out, double *ll_out, double *gamma,
                                    double *log_z, int32_t *active, int32_t *anc, int *flags, const double *exp2t,
                                    hipStream_t stream);
hipError_t launch_adapt(const SmcShape &sh, const DevParticles &p, int n_sound, const rjsmc_prior &pr,
                        double *factors, hipStream_t stream);

// Used slots of a particle archive: slot h is columns h n .. h n + n - 1 of pop (n the
// current population's size), ll likewise, gamma [slot][n_sound], log_z [slot][n_sound][M].
constexpr int kMaxArchive = RJSMC_MAX_ARCHIVE;
struct ArchiveView {
  DevParticles pop;
  const double *ll = nullptr, *gamma = nullptr, *log_z = nullptr;
  int n_used = 0;
};
hipError_t launch_adapt_recycled(const SmcShape &sh, const DevParticles &p, const double *ll, const double *gamma,
                                 const double *log_z, int n_sound, const ArchiveView &ar, const rjsmc_prior &pr,
                                 double *factors, hipStream_t stream);
hipError_t launch_archive_store(const DevParticles &src, const double *ll, const double *gamma, const double *log_z,
                                int n_sound, int n_models, const DevParticlesW &dst, double *ll_dst, double *gamma_dst,
                                double *log_z_dst, int slot, int rows_c, int rows_m, int rows_zm, hipStream_t stream);
hipError_t launch_draw_types(const rjsmc_mutate_args &a, int move, const DevParticles &state, int kc, int km,
                             int32_t *mask, int32_t *type, const int32_t *active, const int32_t *gvalid,
                             hipStream_t stream);
// draw = true: the kernel also draws the move types (runs without gradient moves, which
// need the types before the current-state gradients)
hipError_t launch_propose(const SmcShape &sh, const rjsmc_mutate_args &a, int move, const DevParticles &state,
                          const DevParticlesW &prop, int32_t *mask, int32_t *type, const double *gamma,
                          const DevParticles *grad_cur, int32_t *gvalid, double *lq, const int32_t *active,
                          bool draw, hipStream_t stream);
// Decision of sweep move_prev and proposal of sweep move in one launch (no gradient moves).
hipError_t launch_accept_propose(const SmcShape &sh, const rjsmc_mutate_args &a, int move_prev, int move,
                                 const DevParticlesW &state, double *ll, const DevParticlesW &prop,
                                 const double *ll_prop, int32_t *mask, int32_t *type, const double *gamma,
                                 int64_t *stats, double *lq, const int32_t *active, hipStream_t stream);
hipError_t launch_accept(const SmcShape &sh, const rjsmc_mutate_args &a, int move, const DevParticlesW &state,
                         double *ll, const DevParticles &prop, const double *ll_prop, const int32_t *mask,
                         const int32_t *type, const double *gamma, const DevParticlesW *grad_cur,
                         const DevParticles *grad_prop, int32_t *gvalid, int64_t *stats, const double *lq,
                         hipStream_t stream);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t stream);

// Per-particle scratch of a mutation sweep (and of a layer-sorted forward launch): the
// context's workspace, or the library's static device scratch (noalloc.hip).
struct MutateWorkspace {
  int32_t *mask = nullptr, *type = nullptr, *gvalid = nullptr, *perm = nullptr;
  int *cnt = nullptr;       // 2 kMaxLayers counting-sort counters
  double *lq = nullptr;
  int64_t n = 0;            // particles it holds
  double *rim = nullptr;    // spread evaluation terms for rim_n particles (may be absent)
  int32_t *rim_layers = nullptr;
  int64_t rim_n = 0;
};
// Looks up, once per device and with that device current, the address of the static
// scratch on `device` (hipGetSymbolAddress); later calls return at once.
hipError_t static_scratch_init(int device);
// The static scratch of `device` (false if static_scratch_init has not succeeded there).
bool static_scratch(int device, MutateWorkspace *ws);
// Why the static scratch of `device` is unavailable (hipSuccess if it is available).
hipError_t static_scratch_status(int device);

// Host-side construction of the frequency-to-time matrix (host.cpp).
void build_time_kernel(const double *freq_hz, int n_freq, const double *t_open,
                       const double *t_close, int n_gate, double *K_out);

}  // namespace rjsmc

struct rjsmc_ctx {
  int device;
  int kmax_cond, kmax_charg;
  int precision;
  double z_max;
  rjsmc::DevSystem dev;
  double *K_host;   // [n_gate][n_freq]
  int32_t *work_mask;   // [work_n] mutate scratch: proposal validity
  int32_t *work_type;   // [work_n] mutate scratch: move type
  int32_t *work_gvalid; // [work_n] mutate scratch: the current state's gradient is up to date
  double *work_lq;      // [work_n] mutate scratch: log proposal correction of an adaptive birth/death
  int32_t *work_perm;   // [work_n] evaluation order by layer capacity
  int *work_cnt;        // [2 kMaxLayers] counting-sort scratch
  int64_t work_n;
  double *work_rim;         // [work_rim_n] slots of spread evaluation terms
  int32_t *work_rim_layers; // [work_rim_n] layer counts of the spread evaluation
  int64_t work_rim_n;       // min(work_n, the spread launch limit)
  rjsmc_tuning tuning;  // forward tile shape
  size_t lds_limit;     // LDS bytes one workgroup may use on this device
  int n_cu;             // compute units of the device
};
