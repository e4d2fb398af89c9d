"""Oracle: Algorithm 1 (adaptive reversible-jump static SMC) over the EM forward model.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Plain Python, written from the paper's Algorithm 1 (Section 3.2) with the oracle's own
primitives: the forward model and likelihood of `em` (Section 2, Section 2.3.2), and the
prior draw, temperature bisection, re-weighting, within-model resampling, proposal
factors and RJ-MCMC sweeps of `smc`.  For every sounding (an independent 1-D inversion)
the steps are, in the paper's order:

  initialise the particles from the prior (model counts, then parameters); their
  within-model weights are uniform; gamma_0 = 0 and Z_0,k = 1;
  while gamma_t != 1:
      t <- t + 1;
      choose gamma_t by bisection so that the total effective sample size is alpha N
      (Section 3.2.1), re-weight (evidence update) and re-sample within each model;
      adapt the within-model proposal of every model to the re-sampled particles (the
      principal directions of their sample covariance, Section 3.2.2);
      mutate every particle with R RJ-MCMC sweeps (Appendix E.1) targeting
      L^gamma_t x prior.

Readings (beyond those of `smc`): the number of sweeps R is fixed (the configuration's
R = 5; the adaptive count of Section 3.2.3 is checked separately), the within-model
step is the fixed scale `rw_scale` along a principal direction, and a sounding whose
temperature has reached 1 is neither re-weighted nor mutated again.  The random numbers
are Philox4x32-10 counters: particle i (its index over all soundings) at step t and
sweep r uses (i, t, r, slot); the resampling of model k of sounding s at step t uses
(s, t, k, 2^31); the prior draw of particle i uses (i, 0, slot, 2^30).
"""
import numpy as np

from . import em
from . import smc


def _copy(p):
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in p.items()}


def gradient_vector(system, K, d, p, i):
    """(ll, d ll / d theta) of particle i for data d, the gradient in the order of the
    paper's parameter vector (Section 2.3.1), by the oracle's forward-mode tangents."""
    one = {k: np.ascontiguousarray(v[..., [i]]) for k, v in p.items() if isinstance(v, np.ndarray)}
    one["layout"] = p["layout"]
    ll, g = em.loglik_grad(one, system, K, d)
    names = em.particle_params(one, 0)
    return ll[0], np.array([g[n][0] if r is None else g[n][r, 0] for n, r in names])


def proposal_factors(p, n_sound, n_per_sound, kc, km, pr):
    """Colouring factor of every (sounding, model) from the current population
    (smc.proposal_factor: principal directions of the members' sample covariance, or the
    prior-scaled diagonal for too few members)."""
    models = smc.model_id(np.asarray(p["kappa"]), np.asarray(p["lambda_"]), km)
    out = {}
    for s in range(n_sound):
        base = s * n_per_sound
        for m in range(smc.n_models(kc, km)):
            k, l = m // (km + 1), m % (km + 1)
            members = np.nonzero(models[base:base + n_per_sound] == m)[0] + base
            out[(s, m)] = smc.proposal_factor(p, members, k, l, pr)
    return out


def run(system, K, y_obs, n_sound, n_per_sound, pr, seed, *, alpha=0.5, n_moves=5,
        move_prob=(1, 1, 1, 1, 1, 1, 1, 0), z_move_sd=None, rw_scale=2.38, mala_eps=0.8,
        max_steps=1000, on_step=None, population=None, loglik=None):
    """Algorithm 1 for n_sound soundings of n_per_sound particles (y_obs [n_sound][n_gate]).

    population: the initial population (default: the prior draw smc.init_population with
    `seed`).  loglik(pop, i, s): a stand-in log-likelihood of particle i of sounding s
    (default: the EM model of `em` with the sounding's data).  on_step(t, rec) is called after every step with copies of:
      gamma [S], log_z [S][M] after the re-weighting of step t, anc [n] (global
      indices; particle j of the re-sampled population is a copy of anc[j]), active [S]
      (soundings re-weighted at this step), pop and ll after the mutation, stats
      [2][8] (proposed / accepted per move type in this step), margins (particle,
      sweep, accept margin) of every decided proposal.
    If on_step returns a (pop, ll) pair, the run continues from that population.
    Returns (gamma, log_z, pop, ll, steps)."""
    kc, km = int(system["kmax_cond"]), int(system["kmax_charg"])
    n = n_sound * n_per_sound
    y_obs = np.asarray(y_obs, dtype=np.float64).reshape(n_sound, -1)
    M = smc.n_models(kc, km)
    if z_move_sd is None:
        z_move_sd = 0.05 * pr["z_max"]
    p = smc.init_population(seed, n, kc, km, pr) if population is None else _copy(population)
    sound = lambda i: int(i) // n_per_sound
    if loglik is None:
        ll = np.concatenate([em.loglik(p, system, K, y_obs[s], range(s * n_per_sound, (s + 1) * n_per_sound))
                             for s in range(n_sound)])
        loglik_fn = lambda pp, i: em.loglik(pp, system, K, y_obs[sound(i)], [i])[0]
    else:
        ll = np.array([loglik(p, i, sound(i)) for i in range(n)], dtype=np.float64)
        loglik_fn = lambda pp, i: loglik(pp, i, sound(i))
    gamma = np.zeros(n_sound)
    log_z = np.zeros((n_sound, M))
    q = dict(move_prob=np.asarray(move_prob, dtype=np.float64), z_move_sd=z_move_sd, rw_scale=rw_scale,
             mala_eps=mala_eps)
    grad_fn = lambda pp, i: gradient_vector(system, K, y_obs[sound(i)], pp, i)
    t = 0
    while t < max_steps and np.any(gamma < 1.0):
        t += 1
        active = gamma < 1.0
        # choose gamma_t, re-weight and re-sample within each model
        gamma, log_z, anc = smc.reweight_resample(ll, p["kappa"], p["lambda_"], kc, km, gamma, log_z, alpha,
                                                  seed, t, n_per_sound)
        p = smc.gather(p, anc)
        ll = ll[anc].copy()
        # adapt the within-model proposals to the re-sampled particles
        F = proposal_factors(p, n_sound, n_per_sound, kc, km, pr)
        factor_of = lambda i: F[(sound(i), smc.model_id(int(p["kappa"][i]), int(p["lambda_"][i]), km))]
        # mutate the particles of the soundings re-weighted at this step
        idx = [i for i in range(n) if active[sound(i)]]
        stats, margins = smc.mutate(p, ll, loglik_fn, lambda i: gamma[sound(i)], t, seed, q, pr, kc, km,
                                    factor_of, n_moves, grad_fn=grad_fn, indices=idx)
        if on_step is not None:
            rec = dict(gamma=gamma.copy(), log_z=log_z.copy(), anc=anc.copy(), active=active.copy(),
                       pop=_copy(p), ll=ll.copy(), stats=stats.copy(), margins=list(margins))
            new = on_step(t, rec)
            if new is not None:
                p, ll = _copy(new[0]), np.array(new[1], dtype=np.float64)
    return gamma, log_z, p, ll, t
