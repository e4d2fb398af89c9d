"""Pins of the SMC oracle: published RNG vectors, closed-form evidence of a conjugate
two-model problem, invariants of the tempering bisection and of systematic
resampling, and prior invariance of the RJ-MCMC proposals."""
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import smc
from paper_2109_00661_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
PR = W.PRIOR


def test_philox_known_answers():
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        assert smc.philox4x32_10(v[:4], v[4:6]) == v[6:10]


def test_uniforms_and_normals():
    u = np.array([smc.uniform_pair(7, i, 3, 1, 0) for i in range(20000)]).ravel()
    assert u.min() > 0 and u.max() < 1
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    z = np.array([smc.normal_pair(*smc.uniform_pair(7, i, 3, 2, 0)) for i in range(20000)]).ravel()
    assert stats.kstest(z, "norm").pvalue > 1e-3


# ------------------------------------------------------------------------- tempering
def test_tess_limits_and_monotone():
    rng = np.random.default_rng(0)
    ll = rng.normal(-50, 20, 300)
    models = rng.integers(0, 6, 300)
    assert abs(smc.tess(ll, models, 0.0) - 300) < 1e-9
    vals = [smc.tess(ll, models, g) for g in np.linspace(0, 1, 60)]
    assert all(b <= a + 1e-9 for a, b in zip(vals, vals[1:]))


def test_bisection_brackets_target():
    rng = np.random.default_rng(1)
    ll = rng.normal(-500, 200, 512)
    models = rng.integers(0, 8, 512)
    for gamma in (0.0, 0.3, 0.97):
        dg = smc.next_dgamma(ll, models, gamma, 0.5)
        assert 0 < dg <= 1 - gamma
        assert smc.tess(ll, models, dg) >= 0.5 * 512
        if dg < 1 - gamma:
            assert smc.tess(ll, models, dg + 2.0 ** -50 * (1 - gamma)) < 0.5 * 512


def test_constant_likelihood_single_step():
    ll = np.full(64, -3.25)
    kap = np.repeat([0, 1, 2, 3], 16)
    lam = np.zeros(64, dtype=int)
    g, lz, anc = smc.reweight_resample(ll, kap, lam, 4, 3, np.zeros(1), np.zeros((1, 20)), 0.5, 9, 1)
    assert g[0] == 1.0
    present = [smc.model_id(k, 0, 3) for k in range(4)]
    for m in present:
        assert abs(lz[0, m] - (-3.25)) < 1e-14
    # models without particles: empty sum of incremental weights, estimate 0
    assert all(lz[0, m] == -np.inf for m in range(20) if m not in present)
    assert np.array_equal(anc, np.arange(64))          # equal weights: every particle once


# -------------------------------------------------------------------- resampling
def test_systematic_counts_within_floor_ceil():
    rng = np.random.default_rng(2)
    for trial in range(20):
        N = 200
        models = rng.integers(0, 5, N)
        W_ = np.zeros(N)
        for k in range(5):
            sel = models == k
            w = rng.exponential(1.0, sel.sum()) ** 3
            W_[sel] = w / w.sum()
        U = [int(rng.integers(0, 2 ** 53)) for _ in range(5)]
        anc = smc.systematic_within_model(W_, models, range(5), U)
        assert np.all(models[anc] == models)           # within-model
        counts = np.bincount(anc, minlength=N)
        for k in range(5):
            sel = np.nonzero(models == k)[0]
            nk = len(sel)
            expct = nk * W_[sel]
            assert np.all(counts[sel] >= np.floor(expct - 1e-9)) and np.all(counts[sel] <= np.ceil(expct + 1e-9))
            assert counts[sel].sum() == nk


# --------------------------------------------------------------------- evidence (P12)
@pytest.mark.slow
def test_conjugate_two_model_evidence():
    rng = np.random.default_rng(3)
    x = np.linspace(-1, 1, 8)
    y = 0.8 * x + 0.3 * x ** 2 + rng.normal(0, 0.3, 8)    # posterior odds about 0.71 : 0.29
    toy = smc.NestedLinearGaussian(x, y, 0.09, 1.0)
    exact = np.array([toy.log_evidence(0), toy.log_evidence(1)])
    post = np.exp(exact - np.logaddexp(*exact))
    assert 0.2 < post[1] < 0.8
    lzs, fr = [], []
    for seed in range(24):
        lz, counts = smc.toy_rjsmc(toy, 300, 0.5, seed, n_moves=10)
        lzs.append(lz)
        fr.append(counts / counts.sum())
    lzs, fr = np.array(lzs), np.array(fr)
    ratio = np.exp(lzs - exact[None, :])                 # unbiased for 1
    se = ratio.std(axis=0, ddof=1) / math.sqrt(len(ratio))
    assert np.all(np.abs(ratio.mean(axis=0) - 1) <= 3 * se + 0.02), (ratio.mean(axis=0), se)
    se_f = fr.std(axis=0, ddof=1) / math.sqrt(len(fr))
    assert np.all(np.abs(fr.mean(axis=0) - post) <= 3 * se_f + 0.01), (fr.mean(0), post)


def test_toy_tempered_evidence_closed_form_consistency():
    """The closed form at g -> 0 is 0 and is concave increasing along the path's log."""
    x = np.linspace(-1, 1, 8)
    toy = smc.NestedLinearGaussian(x, np.sin(3 * x), 0.05, 2.0)
    assert abs(toy.log_evidence(1, 0.0)) < 1e-12
    # d/dg log Z_g = E_g[log L] and it is non-decreasing in g
    gs = np.linspace(0.05, 1, 20)
    lz = np.array([toy.log_evidence(1, g) for g in gs])
    d = np.diff(lz) / np.diff(gs)
    assert np.all(np.diff(d) >= -1e-6)


# ------------------------------------------------------------------ prior and mutation
def test_prior_draw_support():
    p = smc.init_population(5, 500, 4, 3, PR)
    assert set(np.unique(p["kappa"])) == set(range(5)) and set(np.unique(p["lambda_"])) == set(range(4))
    for i in range(500):
        th = smc.param_vector(p, i)
        assert smc.in_support(th, int(p["kappa"][i]), int(p["lambda_"][i]), PR)


def _q(probs=None):
    return dict(move_prob=np.array(probs if probs is not None else [1, 1, 1, 1, 1, 1, 1, 0], float),
                z_move_sd=0.05 * PR["z_max"], rw_scale=2.38)


def test_mutation_preserves_the_prior_at_zero_temperature():
    """With gamma = 0 the target is the prior: after many RJ moves the model counts stay
    uniform and the depths and properties stay uniform (detailed balance of the
    birth/death/move/within proposals with respect to the prior)."""
    n = 3000
    p = smc.init_population(11, n, 4, 3, PR)
    ll = np.zeros(n)
    fac = {}

    def factor(i):
        key = (int(p["kappa"][i]), int(p["lambda_"][i]))
        if key not in fac:
            fac[key] = np.diag(0.3 * smc.prior_sd(key[0], key[1], PR))
        return fac[key]

    st, _ = smc.mutate(p, ll, lambda pp, i: 0.0, lambda i: 0.0, 1, 13, _q(), PR, 4, 3, factor, 6)
    assert st[1].sum() > 0.5 * st[0].sum()
    ck = np.bincount(p["kappa"], minlength=5)
    cl = np.bincount(p["lambda_"], minlength=4)
    assert stats.chisquare(ck).pvalue > 1e-3 and stats.chisquare(cl).pvalue > 1e-3
    zs = np.concatenate([p["z_cond"][:k, i] for i, k in enumerate(p["kappa"])])
    assert stats.kstest(zs / PR["z_max"], "uniform").pvalue > 1e-3
    phs = np.concatenate([[p["phi_b"][i]] + list(p["phi"][:k, i]) for i, k in enumerate(p["kappa"])])
    assert stats.kstest((phs - PR["phi_lo"]) / (PR["phi_hi"] - PR["phi_lo"]), "uniform").pvalue > 1e-3


def test_birth_inserts_sorted_and_death_removes():
    p = W.truth_three_layer()
    zc, ph = p["z_cond"][:2, 0], p["phi"][:2, 0]
    z2, v2 = smc._birth(zc, ph, 30.0, -0.5, 4)
    assert list(z2) == [20.0, 30.0, 40.0] and list(v2) == [-1.0, -0.5, -3.0]
    assert smc._birth(np.arange(4.0), np.zeros(4), 1.5, 0.0, 4) is None


def test_acceptance_uses_tempered_ratio():
    """A particle whose proposals all have ll' = ll - 10 is accepted with probability
    exp(-10 gamma)."""
    n = 4000
    p = smc.init_population(17, n, 4, 3, PR)
    for g in (0.05, 0.2):
        pp = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in p.items()}
        ll = np.zeros(n)
        st, _ = smc.mutate(pp, ll, lambda q, i: float(ll[i]) - 10.0, lambda i: g, 2, 21, _q([0, 0, 0, 0, 0, 0, 1, 0]),
                           PR, 4, 3, lambda i: np.diag(1e-6 * smc.prior_sd(int(pp["kappa"][i]), int(pp["lambda_"][i]), PR)), 1)
        rate = st[1, 6] / st[0, 6]
        assert abs(rate - math.exp(-10 * g)) < 4 * math.sqrt(math.exp(-10 * g) / n) + 0.01


def test_mala_log_q_ratio_matches_gaussian_densities():
    """The simplified Langevin correction equals the ratio of the two Gaussian proposal
    densities N(theta; theta' + eps^2/2 S g', eps^2 S) / N(theta'; theta + eps^2/2 S g,
    eps^2 S)."""
    from scipy.stats import multivariate_normal as mvn
    rng = np.random.default_rng(4)
    for d in (3, 7, 11):
        F = rng.standard_normal((d, d)) + 2 * np.eye(d)
        S = F @ F.T
        eps, gamma = 0.37, 0.6
        theta = rng.standard_normal(d)
        g0, g1 = rng.standard_normal(d), rng.standard_normal(d)
        xi = rng.standard_normal(d)
        th1 = smc.mala_propose(theta, g0, gamma, F, eps, xi)
        fwd = mvn.logpdf(th1, theta + 0.5 * eps ** 2 * S @ (gamma * g0), eps ** 2 * S)
        rev = mvn.logpdf(theta, th1 + 0.5 * eps ** 2 * S @ (gamma * g1), eps ** 2 * S)
        assert abs(smc.mala_log_q_ratio(xi, g0, g1, gamma, F, eps) - (rev - fwd)) < 1e-9


def test_mala_preserves_the_prior_at_zero_temperature():
    n = 2000
    p = smc.init_population(23, n, 4, 3, PR)
    ll = np.zeros(n)
    q = dict(move_prob=np.array([0, 0, 0, 0, 0, 0, 0, 1], float), z_move_sd=15.0, rw_scale=2.38, mala_eps=0.8)
    fac = lambda i: np.diag(0.3 * smc.prior_sd(int(p["kappa"][i]), int(p["lambda_"][i]), PR))
    grad = lambda pp, i: (0.0, np.zeros(3 + 2 * int(pp["kappa"][i]) + 2 * int(pp["lambda_"][i])))
    st, _ = smc.mutate(p, ll, lambda pp, i: 0.0, lambda i: 0.0, 1, 29, q, PR, 4, 3, fac, 8, grad_fn=grad)
    assert st[1, 7] > 0.3 * st[0, 7]
    phs = np.array([p["phi_b"][i] for i in range(n)])
    assert stats.kstest((phs - PR["phi_lo"]) / (PR["phi_hi"] - PR["phi_lo"]), "uniform").pvalue > 1e-3
    cs = (p["c"] - PR["c_lo"]) / (PR["c_hi"] - PR["c_lo"])
    assert stats.kstest(cs, "uniform").pvalue > 1e-3


# ----------------------------------------------------------------- posterior summaries
def _population(counts_kl, kc=4, km=3, seed=0):
    """Decoupled population with the given (kappa, lambda) per particle."""
    from paper_2109_00661_amd import workloads as W
    n = len(counts_kl)
    p = W.prior_population(n, kc, km, seed=seed)
    rng = np.random.default_rng(seed + 1)
    for i, (k, l) in enumerate(counts_kl):
        p["kappa"][i], p["lambda_"][i] = k, l
        p["z_cond"][:, i] = np.concatenate([np.sort(rng.uniform(0, 300, k)), np.zeros(kc - k)])
        p["z_charg"][:, i] = np.concatenate([np.sort(rng.uniform(0, 300, l)), np.zeros(km - l)])
    return p


def test_bfipd_is_one_when_the_posterior_equals_the_prior():
    """Every model equally populated: posterior model probabilities equal the uniform
    prior, so the Bayes factor of any grouping is 1."""
    kl = [(k, l) for k in range(5) for l in range(4)] * 3
    out = smc.posterior_summary(_population(kl), 4, 3, 1, [])
    assert out["model_count"][0].tolist() == [3] * 20
    assert abs(out["log_bfipd"][0]) < 1e-14


def test_bfipd_limits_and_posterior_odds():
    kl = [(1, 2)] * 10
    assert smc.posterior_summary(_population(kl), 4, 3, 1, [])["log_bfipd"][0] == np.inf
    kl = [(3, 0)] * 10
    assert smc.posterior_summary(_population(kl), 4, 3, 1, [])["log_bfipd"][0] == -np.inf
    # a Bayes factor is posterior odds over prior odds; prior odds of chargeability = 15:5
    rng = np.random.default_rng(4)
    kl = list(zip(rng.integers(0, 5, 300), rng.integers(0, 4, 300)))
    out = smc.posterior_summary(_population(kl), 4, 3, 1, [])
    pc = np.mean([l >= 1 for _, l in kl])
    assert abs(out["log_bfipd"][0] - (np.log(pc / (1 - pc)) - np.log(15 / 5))) < 1e-12


def test_profiles_match_the_merged_stack():
    """Depth profiles from interface counting equal the merged layer stack of the forward
    model (layer tops from cumulative thicknesses), particle by particle."""
    from oracle import em
    rng = np.random.default_rng(9)
    kl = list(zip(rng.integers(0, 5, 40), rng.integers(0, 4, 40)))
    p = _population(kl, seed=9)
    depths = np.linspace(0.5, 299.5, 37)
    out = smc.posterior_summary(p, 4, 3, 40, depths)      # one particle per sounding
    for i in range(40):
        sig, ms, thick = em.merged_stack(p, i)
        tops = np.concatenate([[0.0], np.cumsum(thick)])
        layer = np.searchsorted(tops, depths, side="right") - 1
        np.testing.assert_allclose(out["mean_log10_sigma"][i], np.log10(np.array(sig))[layer], rtol=0, atol=1e-12)
        np.testing.assert_array_equal(out["mean_m"][i], np.array(ms)[layer])
        np.testing.assert_array_equal(out["p_chargeable"][i], (np.array(ms)[layer] > 0).astype(float))


# ------------------------------------------------------------- adaptive mutation count
def test_mutation_count_is_the_smallest_sufficient_count():
    """R is the smallest number of sweeps with (1 - p_min)^R <= c (brute force)."""
    rng = np.random.default_rng(12)
    for _ in range(2000):
        acc = rng.uniform(0.001, 0.999, rng.integers(1, 6)).tolist()
        c = 10 ** rng.uniform(-4, -0.5)
        p = min(acc)
        R = 1
        while (1 - p) ** R > c:
            R += 1
        assert smc.mutation_count(acc, c, 10 ** 6) == R
    assert smc.mutation_count([0.5, 0.0], 0.01, 77) == 77
    assert smc.mutation_count([1.0], 0.01, 77) == 1
    assert smc.mutation_count([1e-6], 0.01, 50) == 50
    assert smc.mutation_count([0.5], 0.01, 100) == 7                 # 0.5^7 < 0.01 < 0.5^6


@pytest.mark.slow
def test_conjugate_evidence_with_adaptive_mutation_count():
    """Adapting R from the acceptance rates keeps the evidence estimate unbiased."""
    rng = np.random.default_rng(3)
    x = np.linspace(-1, 1, 8)
    y = 0.8 * x + 0.3 * x ** 2 + rng.normal(0, 0.3, 8)
    toy = smc.NestedLinearGaussian(x, y, 0.09, 1.0)
    exact = np.array([toy.log_evidence(0), toy.log_evidence(1)])
    lzs = np.array([smc.toy_rjsmc(toy, 300, 0.5, seed, n_moves=3, adapt_c=0.05, r_max=20)[0] for seed in range(16)])
    ratio = np.exp(lzs - exact[None, :])
    se = ratio.std(axis=0, ddof=1) / math.sqrt(len(ratio))
    assert np.all(np.abs(ratio.mean(axis=0) - 1) <= 3 * se + 0.02), (ratio.mean(axis=0), se)


def test_driver_mutation_count_matches_the_oracle():
    from paper_2109_00661_amd.rjsmc import mutation_count
    rng = np.random.default_rng(13)
    for _ in range(2000):
        acc = rng.uniform(0.0, 1.0, rng.integers(1, 8)).tolist()
        if rng.uniform() < 0.05:
            acc.append(0.0)
        c, r_max = 10 ** rng.uniform(-4, -0.3), int(rng.integers(1, 300))
        assert mutation_count(acc, c, r_max) == smc.mutation_count(acc, c, r_max)


# ------------------------------------------------------------- step-size bisection
def test_scale_bisection_finds_the_gaussian_random_walk_scale():
    """For a standard normal target, a random walk x + s xi is accepted at rate
    (2/pi) arctan(2/s); bisecting to 0.44 must give s = 2/tan(0.22 pi) ~ 2.42."""
    rate = lambda s: 2.0 / math.pi * math.atan(2.0 / s)
    lo, hi = math.log(0.05), math.log(20.0)
    s = math.exp(0.5 * (lo + hi))
    for _ in range(40):
        tried = 10 ** 9
        lo, hi, s = smc.scale_bisection(lo, hi, tried, round(rate(s) * tried), 0.44)
    assert abs(s - 2.0 / math.tan(0.22 * math.pi)) < 1e-6
    assert smc.scale_bisection(0.0, 1.0, 0, 0, 0.44) == (0.0, 1.0, math.exp(0.5))   # no trials: unchanged


def test_trial_proposals_keep_the_population(system, K_oracle, truth_data):
    from oracle import em
    p = smc.init_population(8, 24, PR["kmax_cond"], PR["kmax_charg"], PR)
    ll = em.loglik(p, system, K_oracle, truth_data)
    p0 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in p.items()}
    ll0 = ll.copy()
    q = dict(move_prob=np.array([0, 0, 0, 0, 0, 0, 1, 0], float), z_move_sd=15.0, rw_scale=lambda i: 0.5 + 0.1 * i)
    F = lambda i: np.diag(0.05 * smc.prior_sd(int(p["kappa"][i]), int(p["lambda_"][i]), PR))
    st, margins = smc.mutate(p, ll, lambda pp, i: em.loglik(pp, system, K_oracle, truth_data, [i])[0],
                             lambda i: 0.3, 4, 99, q, PR, PR["kmax_cond"], PR["kmax_charg"], F, 1, trial=2)
    for k, v in p0.items():
        if isinstance(v, np.ndarray):
            assert np.array_equal(p[k], v), k
    assert np.array_equal(ll, ll0)
    assert st[0, 6] == 24 and st[1, 6] == sum(1 for _, _, m in margins if 0 < m < np.inf)


# ------------------------------------------------------------------- particle recycling
def _norm_w(lw):
    w = np.exp(lw - np.max(lw))
    return w / w.sum()


def test_recycled_factor_of_one_population_is_the_plain_factor():
    """A pool holding only the current population has equal weights: the recycled factor
    is the factor of the sample covariance (Section 3.2.2)."""
    p = smc.init_population(4, 600, PR["kmax_cond"], PR["kmax_charg"], PR)
    models = smc.model_id(p["kappa"], p["lambda_"], PR["kmax_charg"])
    k, l = 2, 1
    members = np.nonzero(models == k * (PR["kmax_charg"] + 1) + l)[0]
    thetas = np.array([smc.param_vector(p, i) for i in members])
    ll = np.random.default_rng(0).normal(-80, 5, len(members))
    lw = smc.recycled_log_weights(ll, [0.3], [-12.0], [len(members)], 0.3)
    np.testing.assert_allclose(_norm_w(lw), 1.0 / len(members), rtol=1e-12)
    F = smc.recycled_proposal_factor(thetas, lw, k, l, PR)
    F0 = smc.proposal_factor(p, members, k, l, PR)
    np.testing.assert_allclose(F @ F.T, F0 @ F0.T, rtol=0, atol=1e-12 * np.abs(F0 @ F0.T).max())


def test_recycled_weights_with_equal_counts_are_the_papers_weights():
    """With the same number of members from every step the count-weighted mixture gives
    the normalised weights of the paper's nu = L^g_t p / (1/t sum_l L^g_l p / Z_l)."""
    rng = np.random.default_rng(2)
    ll = rng.normal(-40, 15, 500)
    gam = np.array([0.0, 0.01, 0.07, 0.3, 0.55])
    lz = np.array([0.0, -0.4, -2.5, -9.0, -15.0])
    lw = smc.recycled_log_weights(ll, gam, lz, [100] * 5, gam[-1])
    nu = np.exp(gam[-1] * ll) / (np.sum([np.exp(g * ll - z) for g, z in zip(gam, lz)], axis=0) / (len(gam) - 1))
    np.testing.assert_allclose(_norm_w(lw), nu / nu.sum(), rtol=1e-10)


def test_recycled_weights_invariances_and_dead_members():
    rng = np.random.default_rng(3)
    ll = rng.normal(-30, 10, 200)
    ll[5] = -np.inf
    gam, lz, cnt = [0.0, 0.1, 0.4], [0.0, -3.0, -11.0], [50, 20, 130]
    w = _norm_w(smc.recycled_log_weights(ll, gam, lz, cnt, 0.4))
    assert w[5] == 0.0 and np.all(np.isfinite(w))
    # a common shift of every log Z, or a common factor on every count, leaves them alone
    np.testing.assert_allclose(_norm_w(smc.recycled_log_weights(ll, gam, np.array(lz) + 7.0, cnt, 0.4)), w, rtol=1e-12)
    np.testing.assert_allclose(_norm_w(smc.recycled_log_weights(ll, gam, lz, np.array(cnt) * 3, 0.4)), w, rtol=1e-12)
    # steps without members are not mixture components
    np.testing.assert_allclose(_norm_w(smc.recycled_log_weights(ll, gam + [0.2], lz + [-np.inf], cnt + [0], 0.4)),
                               w, rtol=1e-12)


def test_recycled_moments_match_the_tempered_gaussian():
    """Exact draws from the power posteriors of a Gaussian prior and likelihood, with
    unequal counts per step and the closed-form normalising constants: the recycled
    weighted mean and covariance recover the current power posterior.  Plausible
    mistakes (counts dropped, evidence dropped or sign-flipped, gamma_t in the mixture)
    miss it by far more than the tolerance."""
    rng = np.random.default_rng(1)
    d, s0, s = 3, 2.0, 0.5
    m = np.array([1.5, -1.0, 0.5])
    gam = np.array([0.0, 0.002, 0.01, 0.05, 0.25])
    cnt = np.array([30000, 800, 3000, 600, 5000])

    def post(g):
        P = 1.0 / s0 ** 2 + g / s ** 2
        return (g / s ** 2) * m / P, 1.0 / P

    def log_z(g):
        a, b = s0 ** 2, g / s ** 2
        return float(np.sum(-0.5 * np.log1p(a * b) - b * m ** 2 / (2.0 * (1.0 + a * b))))

    X, LL = [], []
    for g, n in zip(gam, cnt):
        mu, v = post(g)
        x = mu + math.sqrt(v) * rng.standard_normal((n, d))
        X.append(x)
        LL.append(-0.5 * np.sum((x - m) ** 2, axis=1) / s ** 2)
    X, LL = np.concatenate(X), np.concatenate(LL)
    lz = np.array([log_z(g) for g in gam])
    mu_t, v_t = post(gam[-1])

    def miss(lw):
        mu, C = smc.weighted_covariance(X, lw)
        return max(np.abs(mu - mu_t).max() / math.sqrt(v_t), np.abs(np.diag(C) / v_t - 1.0).max(),
                   np.abs(C - np.diag(np.diag(C))).max() / v_t)

    assert miss(smc.recycled_log_weights(LL, gam, lz, cnt, gam[-1])) < 0.04
    assert miss(smc.recycled_log_weights(LL, gam, lz, np.ones_like(cnt), gam[-1])) > 0.07
    assert miss(smc.recycled_log_weights(LL, gam, np.zeros_like(lz), cnt, gam[-1])) > 0.07
    assert miss(smc.recycled_log_weights(LL, gam, -lz, cnt, gam[-1])) > 0.07
    assert miss(smc.recycled_log_weights(LL, np.full_like(gam, gam[-1]), lz, cnt, gam[-1])) > 0.07


def test_recycled_weight_of_a_dead_member_without_a_prior_component_is_zero():
    lw = smc.recycled_log_weights(np.array([-np.inf, -3.0]), [0.2, 0.5], [-1.0, -2.0], [4, 4], 0.5)
    assert lw[0] == -np.inf and np.isfinite(lw[1])


def test_recycled_factor_falls_back_when_the_weights_concentrate():
    k, l = 1, 0
    d = 3 + 2 * k
    X = np.random.default_rng(5).normal(size=(40, d))
    lw = np.full(40, -1e3)
    lw[:3] = 0.0                                     # effective sample size 3 <= d = 5
    F = smc.recycled_proposal_factor(X, lw, k, l, PR)
    np.testing.assert_array_equal(F, np.diag(0.1 * smc.prior_sd(k, l, PR)))
    lw[:8] = 0.0
    F = smc.recycled_proposal_factor(X, lw, k, l, PR)
    _, C = smc.weighted_covariance(X[:8], np.zeros(8))
    np.testing.assert_allclose(F @ F.T, np.cov(X[:8], rowvar=False), rtol=1e-12, atol=1e-14)


# -------------------------------------------------------------------- adaptive birth
def _random_factor(d, seed, scale=None):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(d, d)) * (scale if scale is not None else 1.0)
    return np.linalg.qr(A)[0] * rng.uniform(0.05, 0.6, d)[None, :]


def test_zca_row_is_the_symmetric_square_root():
    F = _random_factor(9, 1)
    F[:, 4] = 0.0                                    # a zero direction contributes nothing
    S = np.array([smc.zca_row(F, i) for i in range(9)])
    np.testing.assert_allclose(S, S.T, rtol=0, atol=1e-15)
    np.testing.assert_allclose(S @ S, F @ F.T, rtol=0, atol=1e-14)
    assert np.all(np.linalg.eigvalsh(S) > -1e-15)
    D = np.diag([0.3, 2.0, 0.0, 5.0])
    np.testing.assert_array_equal(np.array([smc.zca_row(D, i) for i in range(4)]), D)


@pytest.mark.parametrize("part", [0, 1])
def test_zca_birth_then_death_is_the_identity(part):
    """The death of the interface a birth inserted, with the same covariance root,
    recovers the smaller state and negates the log proposal correction."""
    rng = np.random.default_rng(7 + part)
    p = smc.init_population(31 + part, 400, 4, 3, PR)
    done = 0
    for i in range(400):
        k, l = int(p["kappa"][i]), int(p["lambda_"][i])
        if (part == 0 and k == 4) or (part == 1 and l == 3):
            continue
        kb, lb = (k + 1, l) if part == 0 else (k, l + 1)
        F = _random_factor(3 + 2 * kb + 2 * lb, i) * 0.05
        theta = smc.param_vector(p, i)
        zn, up = rng.uniform(0, PR["z_max"]), rng.normal()
        res = smc.zca_birth(theta, k, l, part, zn, up, F, PR)
        if res is None or not smc.in_support(res[0], res[1], res[2], PR):
            continue
        th1, k1, l1, lq = res
        z1 = th1[1 + k1:1 + 2 * k1] if part == 0 else th1[1 + 2 * k1 + l1:1 + 2 * k1 + 2 * l1]
        r = int(np.nonzero(z1 == zn)[0][0])
        back = smc.zca_death(th1, k1, l1, part, r, F, PR)
        assert back is not None
        np.testing.assert_allclose(back[0], theta, rtol=1e-12, atol=1e-12)
        assert (back[1], back[2]) == (k, l)
        assert abs(back[3] + lq) < 1e-9
        done += 1
    assert done > 100


def _zca_invariance(monkeypatch=None, drop_jacobian=False, n=3000, sweeps=10):
    p = smc.init_population(17, n, 4, 3, PR)
    ll = np.zeros(n)
    facs = {}

    def factor_of_model(i, k, l):
        if (k, l) not in facs:
            d = 3 + 2 * k + 2 * l
            R = np.random.default_rng(100 + 10 * k + l).normal(size=(d, d))
            facs[(k, l)] = np.diag(smc.prior_sd(k, l, PR)) @ (np.eye(d) + 0.3 * R)
        return facs[(k, l)]

    if drop_jacobian:
        orig = smc.zca_birth

        def no_jacobian(theta, k, l, part, zn, up, F_big, pr):
            res = orig(theta, k, l, part, zn, up, F_big, pr)
            if res is None:
                return None
            jn, js, _ = smc._zca_indices(res[1], res[2], part, 0)
            S = smc.zca_row(F_big, jn)
            return res[0], res[1], res[2], res[3] - math.log(abs(S[jn] - (S[js] if js is not None else 0.0)))
        monkeypatch.setattr(smc, "zca_birth", no_jacobian)
    q = _q([1, 1, 0, 1, 1, 0, 1, 0])
    q["zca"] = True
    q["factor_of_model"] = factor_of_model
    fac = lambda i: factor_of_model(i, int(p["kappa"][i]), int(p["lambda_"][i]))
    st, _ = smc.mutate(p, ll, lambda pp, i: 0.0, lambda i: 0.0, 1, 19, q, PR, 4, 3, fac, sweeps)
    return p, st


@pytest.mark.slow
def test_zca_moves_preserve_the_prior_at_zero_temperature(monkeypatch):
    """With gamma = 0 the adaptive birth and death (with random covariance roots per
    model) leave the prior invariant: uniform model counts and uniform properties and
    depths.  The same chain without the Jacobian term drifts away from it."""
    p, st = _zca_invariance()
    assert st[1, 0] > 0.05 * st[0, 0] and st[1, 1] > 0.05 * st[0, 1]
    ck = np.bincount(p["kappa"], minlength=5)
    cl = np.bincount(p["lambda_"], minlength=4)
    assert stats.chisquare(ck).pvalue > 1e-3 and stats.chisquare(cl).pvalue > 1e-3, (ck, cl)
    zs = np.concatenate([p["z_cond"][:k, i] for i, k in enumerate(p["kappa"])])
    assert stats.kstest(zs / PR["z_max"], "uniform").pvalue > 1e-3
    phs = np.concatenate([[p["phi_b"][i]] + list(p["phi"][:k, i]) for i, k in enumerate(p["kappa"])])
    assert stats.kstest((phs - PR["phi_lo"]) / (PR["phi_hi"] - PR["phi_lo"]), "uniform").pvalue > 1e-3
    ms = np.concatenate([p["m"][:l, i] for i, l in enumerate(p["lambda_"])])
    assert stats.kstest((ms - PR["m_lo"]) / (PR["m_hi"] - PR["m_lo"]), "uniform").pvalue > 1e-3
    p2, _ = _zca_invariance(monkeypatch, drop_jacobian=True)
    ck2 = np.bincount(p2["kappa"], minlength=5)
    cl2 = np.bincount(p2["lambda_"], minlength=4)
    assert min(stats.chisquare(ck2).pvalue, stats.chisquare(cl2).pvalue) < 1e-6, (ck2, cl2)


# ------------------------------------------------------- posterior predictive summaries
def test_posterior_predictive_identical_particles():
    """A population of one repeated response: the PPD is the noise model at that
    response (mean y, sd s(y)), and z is the textbook standardised residual."""
    from oracle import smc
    rng = np.random.default_rng(4)
    y = rng.uniform(-5, 1e4, 20)
    eps_an, eps_mn = np.full(20, 0.1), 0.03
    d = y + rng.standard_normal(20)
    mean, sd, z = smc.posterior_predictive(np.tile(y, (37, 1)), 1, d, eps_an, eps_mn)
    np.testing.assert_allclose(mean[0], y, rtol=1e-14)
    np.testing.assert_allclose(sd[0], np.sqrt(eps_an ** 2 + (eps_mn * y) ** 2), rtol=1e-14)
    np.testing.assert_allclose(z[0], (d - y) / np.sqrt(eps_an ** 2 + (eps_mn * y) ** 2), rtol=1e-12, atol=1e-10)


def test_posterior_predictive_two_members_closed_form():
    from oracle import smc
    y1, y2 = np.array([3.0, -2.0, 100.0]), np.array([1.0, 2.0, 50.0])
    eps_an, eps_mn = np.array([0.5, 0.1, 1.0]), 0.1
    d = np.array([2.5, 0.0, 80.0])
    mean, sd, z = smc.posterior_predictive(np.stack([y1, y2]), 1, d, eps_an, eps_mn)
    s1, s2 = eps_an ** 2 + (eps_mn * y1) ** 2, eps_an ** 2 + (eps_mn * y2) ** 2
    var = ((y1 - y2) / 2) ** 2 + (s1 + s2) / 2
    np.testing.assert_allclose(mean[0], (y1 + y2) / 2, rtol=1e-15)
    np.testing.assert_allclose(sd[0], np.sqrt(var), rtol=1e-14)
    np.testing.assert_allclose(z[0], (d - (y1 + y2) / 2) / np.sqrt(var), rtol=1e-13)


def test_posterior_predictive_matches_replicated_data():
    """Brute force: draw a particle uniformly, then replicated data from the noise model
    at its response; the sample mean and sd of 400,000 replicates match the summaries
    within Monte Carlo error (two soundings, soundings kept apart)."""
    from oracle import smc
    rng = np.random.default_rng(8)
    ng, N = 6, 50
    resp = np.concatenate([rng.normal(10.0, 3.0, (N, ng)), rng.normal(-2.0, 0.5, (N, ng))])
    eps_an, eps_mn = np.full(ng, 0.3), 0.05
    d = np.zeros((2, ng))
    mean, sd, _ = smc.posterior_predictive(resp, 2, d, eps_an, eps_mn)
    R = 400000
    for s in range(2):
        pick = resp[s * N + rng.integers(0, N, R)]
        rep = pick + rng.standard_normal((R, ng)) * np.sqrt(eps_an ** 2 + (eps_mn * pick) ** 2)
        assert np.all(np.abs(rep.mean(axis=0) - mean[s]) <= 5 * sd[s] / np.sqrt(R))
        np.testing.assert_allclose(rep.std(axis=0), sd[s], rtol=0.01)
