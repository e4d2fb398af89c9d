"""Parity at the shape of the synthetic survey: 2,000 soundings x 2,048 particles
(4,096,000 particles; the default capacities, 20 models).  The device processes the whole
batch in one call; the oracle recomputes a sample of soundings (re-weight/re-sample:
each sounding is independent, its random numbers keyed by its own index) and a sample
of particles (mutation: each particle's chain depends only on its own state and
counters).  The population is the device's prior draw (bit-identical to the oracle's,
which draws the sampled particles itself); the data are the oracle's responses of the
survey's station models plus seeded noise.  Mutation is checked with random-walk and
Langevin moves in FP64 and with random-walk moves whose proposal likelihoods use the
FP32 forward model."""

import numpy as np
import pytest

from paper_2109_00661_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PR = W.PRIOR
KC, KM = PR["kmax_cond"], PR["kmax_charg"]
M = (KC + 1) * (KM + 1)
D = 3 + 2 * KC + 2 * KM
S, N = 2000, 2048


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_00661_amd import binding
    return binding


@pytest.fixture(scope="module")
def survey_data(system, K_oracle):
    """Oracle responses of the 2,000 station models plus noise of the noise model."""
    from oracle import em
    truth, body, _, _ = W.survey()
    y = em.forward(truth, system, K_oracle)
    sd = np.sqrt(em.noise_variance(y, system["eps_an"][None, :], system["eps_mn"]))
    noise = np.stack([np.random.default_rng(5000 + i).standard_normal(y.shape[1]) for i in range(S)])
    return y + sd * noise


def test_reweight_resample_survey_shape(B, system):
    from oracle import smc
    ctx = B.Context(system, precision="f64", max_particles=S * N)
    n = S * N
    p = B.empty_device_population(n, KC, KM, N)
    ctx.init_prior(p, PR, 41)
    rng = np.random.default_rng(41)
    ll = -np.abs(rng.standard_cauchy(n)) * 50 - rng.uniform(0, 30, n)
    gamma = rng.uniform(0.0, 0.9, S)
    gamma[::211] = 1.0
    log_z = rng.normal(0, 1, (S, M))
    seed, step = 91, 7
    out = B.empty_device_population(n, KC, KM, N)
    ll_d = torch.as_tensor(ll, device="cuda")
    ll_out = torch.empty_like(ll_d)
    g_d = torch.as_tensor(gamma, device="cuda")
    lz_d = torch.as_tensor(log_z, device="cuda")
    anc = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx.reweight_resample(p, ll_d, out, ll_out, g_d, lz_d, None, anc, 0.5, seed, step, S)
    ctx.check()
    g, lz, a = g_d.cpu().numpy(), lz_d.cpu().numpy(), anc.cpu().numpy()
    kap, lam = p["kappa"].cpu().numpy(), p["lambda_"].cpu().numpy()
    for s in (0, 211, 999, 1337, 1999):
        sl = slice(s * N, (s + 1) * N)
        # the sounding's prior counts from the oracle's own draw
        draws = [smc.prior_draw(41, i, KC, KM, PR) for i in range(s * N, (s + 1) * N)]
        kk = np.array([dr["kappa"] for dr in draws])
        ll_ = np.array([dr["lambda_"] for dr in draws])
        assert np.array_equal(kk, kap[sl]) and np.array_equal(ll_, lam[sl]), s
        if gamma[s] >= 1.0:
            assert g[s] == gamma[s] and np.array_equal(lz[s], log_z[s])
            assert np.array_equal(a[sl], np.arange(s * N, (s + 1) * N))
            continue
        mb = smc.model_id(kk, ll_, KM)
        dg = smc.next_dgamma(ll[sl], mb, gamma[s], 0.5)
        lz_ref, Wt = smc.reweight(ll[sl], mb, dg, log_z[s], range(M))
        g_ref = 1.0 if dg == 1.0 - gamma[s] else gamma[s] + dg
        U = [smc.resample_uniform(seed, s, step, k) for k in range(M)]
        anc_ref = smc.systematic_within_model(Wt, mb, range(M), U) + s * N
        assert abs(g[s] - g_ref) <= 1e-12, s
        fin = np.isfinite(lz_ref)
        assert np.array_equal(fin, np.isfinite(lz[s])), s
        np.testing.assert_allclose(lz[s][fin], lz_ref[fin], rtol=1e-11, atol=1e-11)
        assert np.array_equal(a[sl], anc_ref), s
    # the resampled copy follows the ancestors (a sample of rows)
    rows = np.random.default_rng(1).integers(0, n, 4096)
    for k in ("kappa", "lambda_", "phi_b", "c"):
        src, dst = p[k].cpu().numpy(), out[k].cpu().numpy()
        assert np.array_equal(dst[rows], src[a[rows]]), k
    assert np.array_equal(ll_out.cpu().numpy()[rows], ll[a[rows]])


def _factors(seed):
    """Seeded proposal factors for every (sounding, model): device layout and a lookup."""
    from oracle import smc
    rng = np.random.default_rng(seed)
    dev = np.zeros((S, M, D, D))
    base = {}
    for m in range(M):
        k, l = m // (KM + 1), m % (KM + 1)
        d = 3 + 2 * k + 2 * l
        base[m] = np.diag(0.05 * smc.prior_sd(k, l, PR))
        mix = np.eye(d)[None] + 0.3 * rng.standard_normal((S, d, d))
        Fs = base[m][None] @ mix
        dev[:, m, :d, :d] = np.transpose(Fs, (0, 2, 1))
    return dev


@pytest.mark.parametrize("case", ["fp64_rw", "fp64_langevin", "fp32_rw"])
def test_mutate_survey_shape_sampled(B, system, K_oracle, survey_data, case):
    from oracle import algorithm1 as A1, em, smc
    n = S * N
    prec = "f32" if case == "fp32_rw" else "f64"
    ctx = B.Context(system, precision=prec, max_particles=n)
    p = B.empty_device_population(n, KC, KM, N)
    ctx.init_prior(p, PR, 43)
    y_d = torch.as_tensor(survey_data, device="cuda")
    ll_d = ctx.loglik(p, y_d)
    rng = np.random.default_rng(43)
    # FP32: early-step temperatures, at which the FP32 likelihood error (~1e-4 |ll| for
    # prior particles with |ll| ~ 1e5) moves an accept margin by well under a nat
    gamma = rng.uniform(1e-4, 1e-3, S) if prec == "f32" else rng.uniform(0.001, 0.3, S)
    fdev = _factors(47)
    langevin = case == "fp64_langevin"
    mp = np.array([1, 1, 1, 1, 1, 1, 0, 1] if langevin else [1, 1, 1, 1, 1, 1, 1, 0], float)
    q = dict(move_prob=mp, z_move_sd=0.05 * PR["z_max"], rw_scale=2.38, mala_eps=0.5)
    seed, step, n_moves = 4321, 9, 2
    stats = torch.zeros((2, 8), dtype=torch.int64, device="cuda")
    extra = {}
    if langevin:
        extra = dict(mala_eps=q["mala_eps"], grad_cur=B.empty_device_population(n, KC, KM, N),
                     grad_prop=B.empty_device_population(n, KC, KM, N))
    ctx.mutate(p, ll_d, B.empty_device_population(n, KC, KM, N), torch.empty_like(ll_d),
               torch.as_tensor(gamma, device="cuda"), None, y_d, stats, seed=seed, step=step, n_moves=n_moves,
               n_sound=S, prior=PR, move_prob=mp, z_move_sd=q["z_move_sd"], rw_scale=q["rw_scale"],
               factors=torch.as_tensor(fdev, device="cuda"), **extra)
    ctx.check()
    lld = ll_d.cpu().numpy()
    idx = sorted(set(rng.integers(0, n, 20).tolist()) | {0, n - 1, 1234 * N + 77})
    # the oracle's own prior draw of the sampled particles
    po = W.empty_particles(n, KC, KM)
    for i in idx:
        dr = smc.prior_draw(43, i, KC, KM, PR)
        po["kappa"][i], po["lambda_"][i] = dr["kappa"], dr["lambda_"]
        po["phi_b"][i], po["log10_tau"][i], po["c"][i] = dr["phi_b"], dr["log10_tau"], dr["c"]
        po["z_cond"][:dr["kappa"], i], po["phi"][:dr["kappa"], i] = dr["z_cond"], dr["phi"]
        po["z_charg"][:dr["lambda_"], i], po["m"][:dr["lambda_"], i] = dr["z_charg"], dr["m"]
    llo = np.full(n, np.nan)
    for i in idx:
        llo[i] = em.loglik(po, system, K_oracle, survey_data[i // N], [i])[0]
    fh = lambda i: fdev[i // N, smc.model_id(int(po["kappa"][i]), int(po["lambda_"][i]), KM)].T[
        :3 + 2 * int(po["kappa"][i]) + 2 * int(po["lambda_"][i]), :3 + 2 * int(po["kappa"][i]) + 2 * int(po["lambda_"][i])]
    _, margins = smc.mutate(po, llo, lambda pp, i: em.loglik(pp, system, K_oracle, survey_data[i // N], [i])[0],
                            lambda i: gamma[i // N], step, seed, q, PR, KC, KM, fh, n_moves,
                            grad_fn=lambda pp, i: A1.gradient_vector(system, K_oracle, survey_data[i // N], pp, i),
                            indices=idx)
    got = {k: p[k].cpu().numpy() for k in ("kappa", "lambda_", "phi_b", "phi", "z_cond", "m", "z_charg", "log10_tau",
                                           "c")}
    if prec == "f64":
        near = {i for i, r, mg in margins if abs(mg) < 1e-7}
        tol_state, tol_ll = (1e-12 if not langevin else 1e-10), 1e-9
    else:
        # FP32 proposal likelihoods move a margin by up to ~1e-4 |ll| gamma (the FP32 bound)
        near = {i for i, r, mg in margins if abs(mg) < 1e-3 * gamma[i // N] * max(1.0, abs(llo[i])) + 1e-8}
        tol_state, tol_ll = 1e-12, 1e-3
    ok = [i for i in idx if i not in near]
    assert len(ok) >= len(idx) - 3, (len(ok), len(idx))
    for k in ("kappa", "lambda_"):
        assert np.array_equal(got[k][ok], po[k][ok]), k
    for i in ok:
        np.testing.assert_allclose(smc.param_vector(got, i), smc.param_vector(po, i), rtol=tol_state, atol=tol_state,
                                   err_msg=str(i))
    np.testing.assert_allclose(lld[ok], llo[ok], rtol=tol_ll, atol=tol_ll)
    st = stats.cpu().numpy()
    assert st[0].sum() == n * n_moves and st[1].sum() > 0
    if langevin:
        assert st[0, 7] > 0 and st[1, 7] > 0
