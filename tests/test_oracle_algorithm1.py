"""Pins of the oracle's Algorithm-1 driver over the EM model (oracle/algorithm1.py).

* A constant likelihood makes the first tempering step the full one (TESS = N at every
  increment): gamma = 1 after one step, log Z_k = the constant for every populated model
  (-inf for the empty ones), and every in-support proposal is accepted.
* A likelihood that depends only on the background conductivity, Gaussian with mean -1.5
  and sd 0.1 inside the uniform prior on [-3, 0], has the same evidence in every model,
  Z = int_{-3}^{0} N(x; -1.5, 0.1^2) / 3 dx (closed form): the driver's estimate, the
  product over steps of the mean incremental weights, must match it, the posterior of
  phi_b must be N(-1.5, 0.1^2), and the model probabilities stay at the uniform prior.
* Soundings are independent inversions (Section 2): sounding 0 of a two-sounding run is
  identical to the one-sounding run with the same seed.
"""
import math
import warnings

import numpy as np
import pytest

from paper_2109_00661_amd import workloads as W

PR = W.PRIOR


@pytest.fixture(scope="module")
def sysK():
    from oracle import em
    system = W.system()
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        K = em.make_K(system)
    return system, K


def test_constant_likelihood_one_step(sysK):
    from oracle import algorithm1 as A1, smc
    system, K = sysK
    recs = []
    g, lz, p, ll, steps = A1.run(system, K, np.zeros((2, 20)), 2, 48, PR, 3, loglik=lambda pp, i, s: -7.5,
                                 on_step=lambda t, rec: recs.append(rec))
    assert steps == 1 and np.all(g == 1.0)
    init = smc.init_population(3, 96, 4, 3, PR)
    m0 = smc.model_id(init["kappa"], init["lambda_"], 3)
    for s in range(2):
        present = np.unique(m0[s * 48:(s + 1) * 48])
        assert np.all(lz[s, present] == -7.5)
        absent = np.setdiff1d(np.arange(20), present)
        assert np.all(np.isneginf(lz[s, absent]))
    st = recs[0]["stats"]
    decided = sum(1 for _, _, mg in recs[0]["margins"] if np.isfinite(mg))
    assert st[1].sum() == decided > 0
    assert np.all(ll == -7.5)


def test_background_only_likelihood_exact_evidence(sysK):
    from oracle import algorithm1 as A1, smc
    system, K = sysK
    mu, sd = -1.5, 0.1

    def loglik(pp, i, s):
        x = pp["phi_b"][i]
        return -0.5 * ((x - mu) / sd) ** 2 - math.log(sd * math.sqrt(2.0 * math.pi))

    # exact evidence of every model: the prior density of phi_b is 1/3 on [-3, 0]
    z_exact = (math.erf((0.0 - mu) / (sd * math.sqrt(2))) - math.erf((-3.0 - mu) / (sd * math.sqrt(2)))) / 2 / 3.0
    S, N = 8, 400
    g, lz, p, ll, steps = A1.run(system, K, np.zeros((S, 20)), S, N, PR, 11, loglik=loglik, n_moves=5)
    assert np.all(g == 1.0) and 2 <= steps < 40
    M = lz.shape[1]
    assert np.isfinite(lz).all()
    # marginal evidence sum_k p(k) Z_k (uniform model prior), an unbiased estimate per
    # sounding; its spread over soundings is ~0.13 in log, so the mean of 8 is within
    # 0.15 of the exact value at three standard errors
    z_hat = np.exp(lz).mean(axis=1)
    assert abs(math.log(z_hat.mean()) - math.log(z_exact)) < 0.15, (np.log(z_hat), math.log(z_exact))
    xb = p["phi_b"]
    assert abs(xb.mean() - mu) < 0.02 and abs(xb.std() - sd) < 0.02
    models = smc.model_id(p["kappa"], p["lambda_"], 3)
    freq = np.bincount(models, minlength=M) / (S * N)
    assert np.abs(freq - 1.0 / M).max() < 0.03, freq


def test_soundings_are_independent(sysK):
    from oracle import algorithm1 as A1
    system, K = sysK
    ll_fn = lambda pp, i, s: -0.5 * ((pp["phi_b"][i] + 1.0 + 0.3 * s) / 0.02) ** 2
    one = A1.run(system, K, np.zeros((1, 20)), 1, 40, PR, 5, loglik=ll_fn, max_steps=4)
    two = A1.run(system, K, np.zeros((2, 20)), 2, 40, PR, 5, loglik=ll_fn, max_steps=4)
    assert 2 <= one[4] <= two[4]          # sounding 0 stays unchanged once it reaches gamma = 1
    np.testing.assert_array_equal(one[0], two[0][:1])
    np.testing.assert_array_equal(one[1], two[1][:1])
    for k, v in one[2].items():
        if isinstance(v, np.ndarray):
            np.testing.assert_array_equal(v, two[2][k][..., :40], err_msg=k)
