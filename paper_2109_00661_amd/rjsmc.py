"""Algorithm 1 (adaptive RJSMC) driven through the C ABI.

The loop below only sequences library calls and swaps buffers: initialisation from the
prior, then, until every sounding reaches gamma = 1, re-weight + re-sample, adaptation of
the within-model proposals, and R mutation sweeps.  Every arithmetic step runs in the
HIP library; torch holds the device buffers.
"""
import numpy as np

from . import binding as B
from . import workloads as W

UNIFORM_MOVES = (1, 1, 1, 1, 1, 1, 1, 0)     # birth/death/move x2 partitions + within-model RW
LANGEVIN_MOVES = (1, 1, 1, 1, 1, 1, 0, 1)    # the within-model move is the gradient-informed one
RW_ONLY = (0, 0, 0, 0, 0, 0, 1, 0)           # trial proposals of the step-size bisection
MALA_ONLY = (0, 0, 0, 0, 0, 0, 0, 1)         # trial proposals of the Langevin step bisection


def mutation_count(rates, c, r_max):
    """Sweeps for the next step from the last step's acceptance rates per move type
    (Section 3.2.3): the least R with (1 - p_min)^R <= c, clamped to 1 .. r_max."""
    p = min(rates)
    if p <= 0.0:
        return int(r_max)
    if p >= 1.0:
        return 1
    return int(min(max(np.ceil(np.log(c) / np.log1p(-p)), 1), r_max))


class RJSMCRun:
    """One RJSMC run over n_sound soundings of n_per_sound particles each.

    graph=True captures one whole step (re-weight/re-sample, adapt, R mutation sweeps and
    the device step counter) into a HIP graph per ping-pong direction and replays it, so
    a step costs one graph launch instead of tens of kernel launches from Python."""

    def __init__(self, ctx, n_sound, n_per_sound, y_obs, *, prior=None, alpha=0.5, n_moves=5, seed=0,
                 move_prob=UNIFORM_MOVES, z_move_frac=0.05, rw_scale=2.38, mala_eps=0.8, device="cuda",
                 graph=False, adapt_c=None, r_max=100, tune_scale=False, scale_target=None, n_bisect=6,
                 scale_bracket=None, recycle=0, zca_birth=False):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.S, self.N = n_sound, n_per_sound
        self.n = n_sound * n_per_sound
        self.prior = dict(W.PRIOR) if prior is None else prior
        self.alpha, self.n_moves, self.seed = alpha, n_moves, seed
        self.n_moves0 = n_moves
        self._run_base = 0          # step-counter offset of the current run (see rerun)
        self.move_prob = move_prob
        self.z_move_sd = z_move_frac * self.prior["z_max"]
        self.rw_scale = rw_scale
        self.mala_eps = mala_eps
        kc, km = ctx.kmax_cond, ctx.kmax_charg
        self.M = (kc + 1) * (km + 1)
        self.dmax = 3 + 2 * kc + 2 * km
        nps = n_per_sound if n_sound > 1 else 0
        self.bufs = [B.empty_device_population(self.n, kc, km, nps, device) for _ in range(2)]
        self.lls = [torch.empty(self.n, dtype=torch.float64, device=device) for _ in range(2)]
        self.cur = 0
        self.gamma = torch.zeros(n_sound, dtype=torch.float64, device=device)
        # host copy of gamma for the end-of-loop test (pinned, one copy per step)
        self._gamma_host = torch.empty(n_sound, dtype=torch.float64, pin_memory=torch.cuda.is_available())
        self.log_z = torch.zeros((n_sound, self.M), dtype=torch.float64, device=device)
        self.active = torch.ones(n_sound, dtype=torch.int32, device=device)
        self.anc = torch.empty(self.n, dtype=torch.int32, device=device)
        self.factors = torch.zeros((n_sound, self.M, self.dmax, self.dmax), dtype=torch.float64, device=device)
        self.stats = torch.zeros((2, B.N_MOVES), dtype=torch.int64, device=device)
        self.y_obs = torch.as_tensor(np.asarray(y_obs, dtype=np.float64), device=device).reshape(n_sound, -1)
        self.grads = None
        if move_prob[B.N_MOVES - 1] > 0:
            self.grads = [B.empty_device_population(self.n, kc, km, nps, device) for _ in range(2)]
        self.step = 0
        self.adapt_c, self.r_max = adapt_c, r_max
        # bisection of the within-model step on trial proposals (Section 3.2.2): the random
        # walk's scale toward acceptance 0.44, or, when the within-model move is the
        # gradient-informed one, the Langevin step toward 0.574 (the optimal acceptance of
        # Langevin proposals in high dimension, Roberts & Rosenthal 1998)
        self.tune_langevin = move_prob[B.N_MOVES - 1] > 0 and move_prob[B.N_MOVES - 2] == 0
        if scale_target is None:
            scale_target = 0.574 if self.tune_langevin else 0.44
        if scale_bracket is None:
            scale_bracket = (0.02, 4.0) if self.tune_langevin else (0.05, 20.0)
        self.tune_scale, self.scale_target, self.n_bisect, self.scale_bracket = (tune_scale, scale_target, n_bisect,
                                                                                 scale_bracket)
        self.scale0 = mala_eps if self.tune_langevin else rw_scale
        if tune_scale:
            self.log_lo = torch.zeros(n_sound, dtype=torch.float64, device=device)
            self.log_hi = torch.zeros(n_sound, dtype=torch.float64, device=device)
            self.scale = torch.full((n_sound,), self.scale0, dtype=torch.float64, device=device)
            self.stats_sound = torch.zeros((n_sound, 2), dtype=torch.int64, device=device)
        self.moves_per_step = []
        self._stats_prev = None
        # particle recycling (Section 3.2.4): the proposals adapt to the current population
        # pooled with the populations of up to `recycle` earlier steps (a ring)
        if recycle and graph:
            raise ValueError("particle recycling runs eagerly (the archive slot changes every step)")
        if not 0 <= recycle <= B.MAX_ARCHIVE:
            raise ValueError("recycle must be in 0..%d" % B.MAX_ARCHIVE)
        self.archive = B.DeviceArchive(recycle, self.n, n_sound, kc, km, device) if recycle else None
        # births and deaths by the adaptive construction of Appendix E.2
        self.zca_birth = bool(zca_birth)
        self.use_graph = graph
        self.graphs = None
        self.step_dev = None

    @property
    def state(self):
        return self.bufs[self.cur]

    @property
    def ll(self):
        return self.lls[self.cur]

    def initialise(self):
        self.ctx.init_prior(self.state, self.prior, self.seed)
        self.ctx.loglik(self.state, self.y_obs, out=self.ll)
        if self.archive is not None:
            self.archive.n_used = 0
            self._archive_current()

    def _archive_current(self):
        """Stores the current population (step self.step) in its ring slot."""
        a = self.archive
        self.ctx.archive_store(self.state, self.ll, self.gamma, self.log_z, self.S, a, self.step % a.n_slots)
        a.n_used = min(a.n_used + 1, a.n_slots)

    def _launch_step(self, step_dev=None):
        """Enqueues one iteration of the while-loop of Algorithm 1 (step self.step, or the
        value in step_dev when the kernels run) and flips the ping-pong buffers."""
        nxt = 1 - self.cur
        self.ctx.reweight_resample(self.bufs[self.cur], self.lls[self.cur], self.bufs[nxt], self.lls[nxt], self.gamma,
                                   self.log_z, self.active, self.anc, self.alpha, self.seed, self._run_base + self.step,
                                   self.S,
                                   step_dev=step_dev)
        self.cur = nxt
        if self.archive is not None:
            self.ctx.adapt_recycled(self.state, self.ll, self.gamma, self.log_z, self.S, self.archive, self.prior,
                                    self.factors)
        else:
            self.ctx.adapt(self.state, self.S, self.prior, self.factors)
        common = dict(seed=self.seed, step=self._run_base + self.step, n_sound=self.S, prior=self.prior, z_move_sd=self.z_move_sd,
                      rw_scale=self.rw_scale, factors=self.factors, mala_eps=self.mala_eps, step_dev=step_dev,
                      zca_birth=self.zca_birth)
        grads = dict(grad_cur=self.grads[0] if self.grads else None, grad_prop=self.grads[1] if self.grads else None)
        lang = self.tune_scale and self.tune_langevin
        tuned = dict(rw_scale_dev=self.scale if self.tune_scale and not lang else None,
                     mala_eps_dev=self.scale if lang else None)
        if self.tune_scale:
            # bisection on the within-model step from trial proposals (never kept)
            bis = dict(target=self.scale_target, lo0=self.scale_bracket[0], hi0=self.scale_bracket[1],
                       log_lo=self.log_lo, log_hi=self.log_hi, scale=self.scale, stats_sound=self.stats_sound)
            self.ctx.scale_bisect(self.S, 1, **bis)
            for b in range(1, self.n_bisect + 1):
                # trial sweeps never change the states: the current-state gradients of the
                # first Langevin trial serve the later ones and the sweeps that follow
                self.ctx.mutate(self.state, self.ll, self.bufs[1 - self.cur], self.lls[1 - self.cur], self.gamma,
                                self.active, self.y_obs, None, n_moves=1, move_prob=MALA_ONLY if lang else RW_ONLY,
                                stats_sound=self.stats_sound, trial=b, keep_gradients=lang and b > 1, **tuned,
                                **grads, **common)
                self.ctx.scale_bisect(self.S, 0, **bis)
        self.ctx.mutate(self.state, self.ll, self.bufs[1 - self.cur], self.lls[1 - self.cur], self.gamma, self.active,
                        self.y_obs, self.stats, n_moves=self.n_moves, move_prob=self.move_prob,
                        keep_gradients=lang and self.n_bisect > 0, **tuned, **grads, **common)
        if self.archive is not None:
            self._archive_current()
        if step_dev is not None:
            self.ctx.counter_add(step_dev, 1)

    def _capture(self, start):
        """Captures the step from buffer `start` with the current number of sweeps into a
        graph; the device counter holds the step that a replay runs."""
        torch = self.torch
        if self.step_dev is None:
            self.step_dev = torch.full((1,), self._run_base + self.step + 1, dtype=torch.int32,
                                       device=self.gamma.device)
            self.graphs = {}
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        cur0 = self.cur
        self.cur = start
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            self._launch_step(self.step_dev)
        self.graphs[(start, self.n_moves)] = g
        self.cur = cur0
        torch.cuda.current_stream().wait_stream(side)

    def _adapt_sweeps(self):
        """Next step's number of sweeps from this step's acceptance rates."""
        st = self.stats.cpu().numpy()
        prev = self._stats_prev if self._stats_prev is not None else np.zeros_like(st)
        self._stats_prev = st
        tried, taken = st[0] - prev[0], st[1] - prev[1]
        rates = [taken[t] / tried[t] for t in range(B.N_MOVES) if self.move_prob[t] > 0 and tried[t] > 0]
        if rates:
            self.n_moves = mutation_count(rates, self.adapt_c, self.r_max)

    def advance(self):
        """One iteration of the while-loop of Algorithm 1."""
        self.step += 1
        self.moves_per_step.append(self.n_moves)
        if not self.use_graph:
            self._launch_step()
        else:
            if self.graphs is None or (self.cur, self.n_moves) not in self.graphs:
                self.step -= 1
                self._capture(self.cur)
                self.step += 1
            self.graphs[(self.cur, self.n_moves)].replay()
            self.cur = 1 - self.cur
        if self.adapt_c is not None:
            self._adapt_sweeps()

    def finished(self):
        """Whether every sounding has reached gamma = 1 (one device-to-host copy)."""
        self._gamma_host.copy_(self.gamma)
        return bool((self._gamma_host.numpy() >= 1.0).all())

    def run(self, max_steps=1000):
        self.initialise()
        while self.step < max_steps:
            self.advance()
            if self.finished():
                break
        self.ctx.check()
        return self

    def rerun(self, prior_seed, max_steps=1000):
        """Algorithm 1 again on the same buffers for new soundings' worth of work: a fresh
        prior population drawn with `prior_seed`, gamma, evidence and tallies reset, and
        the captured step graphs replayed as they are.  The kernels' random counters carry
        the step, and the device step counter continues from a new base, so the random
        streams of this run are disjoint from every earlier run's (the captured seed is
        kept).  Processing soundings one run after another this way captures the step
        graphs once."""
        self.gamma.zero_()
        self.log_z.zero_()
        self.active.fill_(1)
        self.stats.zero_()
        self.n_moves = self.n_moves0
        self.moves_per_step = []
        self._stats_prev = None
        self._run_base += 1 << 16
        self.step = 0
        if self.step_dev is not None:
            self.step_dev.fill_(self._run_base + 1)
        if self.tune_scale:
            self.scale.fill_(self.scale0)
            self.stats_sound.zero_()
        self.ctx.init_prior(self.state, self.prior, prior_seed)
        self.ctx.loglik(self.state, self.y_obs, out=self.ll)
        if self.archive is not None:
            self.archive.n_used = 0
            self._archive_current()
        while self.step < max_steps:
            self.advance()
            if self.finished():
                break
        self.ctx.check()
        return self

    def posterior_predictive(self):
        """Posterior predictive mean, sd and standardised data per sounding and gate of the
        current population (device call)."""
        return self.ctx.posterior_predictive(self.state, self.S, self.y_obs)

    def model_probabilities(self):
        """pi_T(k | y) = N_{T,k} / N per sounding (Section 3.2.1), from the model counts of
        the device summary (rjsmc_summarize)."""
        counts = self.ctx.summarize(self.state, self.S)["model_count"]
        return counts.cpu().numpy().astype(np.float64) / self.N
