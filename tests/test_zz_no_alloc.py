"""rjsmc_mutate_noalloc (static device scratch) against rjsmc_mutate (context workspace).

Same inputs through both entry points, through the C ABI: states, log-likelihoods and
move tallies must be bit-identical.  Two calls in a row on the allocation-free entry
point, the second with a smaller population, so that the second runs on scratch left
by the first.  The contexts of the allocation-free calls have no workspace at all
(max_particles = 0), so rjsmc_mutate itself refuses them.  The sweeps use every move
type, gradient-informed moves and adaptive births (every scratch array is used) and a
layer-sorted tile shape (the evaluation order and its counters live in the scratch too)."""
import numpy as np
import pytest

from paper_2109_00661_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PR = W.PRIOR
KC, KM = PR["kmax_cond"], PR["kmax_charg"]
M = (KC + 1) * (KM + 1)
D = 3 + 2 * KC + 2 * KM
KEYS = ("kappa", "lambda_", "phi_b", "phi", "z_cond", "m", "z_charg", "log10_tau", "c")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_00661_amd import binding
    return binding


def _case(B, ctx, n, n_sound, seed, truth_data, noalloc):
    """One mutate call of n particles (n_sound soundings) from a seeded prior draw."""
    nps = n // n_sound
    p = B.empty_device_population(n, KC, KM, nps if n_sound > 1 else 0)
    ctx.init_prior(p, PR, seed)
    y = torch.as_tensor(np.tile(truth_data, (n_sound, 1)), device="cuda")
    ll = ctx.loglik(p, y)
    rng = np.random.default_rng(seed)
    F = np.zeros((n_sound, M, D, D))
    for s in range(n_sound):
        for m in range(M):
            k, l = m // (KM + 1), m % (KM + 1)
            d = 3 + 2 * k + 2 * l
            F[s, m, :d, :d] = 0.05 * (np.eye(d) + 0.2 * rng.standard_normal((d, d)))
    gamma = torch.as_tensor(rng.uniform(0.001, 0.05, n_sound), device="cuda")
    stats = torch.zeros((2, 8), dtype=torch.int64, device="cuda")
    gcur = B.empty_device_population(n, KC, KM, p["n_per_sounding"])
    gprop = B.empty_device_population(n, KC, KM, p["n_per_sounding"])
    scratch = B.empty_device_population(n, KC, KM, p["n_per_sounding"])
    ctx.mutate(p, ll, scratch, torch.empty_like(ll), gamma, None, y, stats, seed=seed + 1, step=3, n_moves=3,
               n_sound=n_sound, prior=PR, move_prob=(1, 1, 1, 1, 1, 1, 1, 1), z_move_sd=15.0, rw_scale=2.38,
               factors=torch.as_tensor(F, device="cuda"), mala_eps=0.3, grad_cur=gcur, grad_prop=gprop,
               zca_birth=True, noalloc=noalloc)
    ctx.check()
    out = {k: p[k].cpu().numpy() for k in KEYS}
    return out, ll.cpu().numpy(), stats.cpu().numpy()


def test_noalloc_matches_workspace_twice_shrinking(B, truth_data):
    sys_ = W.system()
    ref = B.Context(sys_, precision="f64", max_particles=4096)
    bare = B.Context(sys_, precision="f64", max_particles=0)
    ref.set_tuning(4, 1, 1)                 # layer-sorted shape: perm + counters in use
    bare.set_tuning(4, 1, 1)
    for n, n_sound, seed in ((3000, 3, 41), (700, 1, 43)):
        a = _case(B, ref, n, n_sound, seed, truth_data, noalloc=False)
        b = _case(B, bare, n, n_sound, seed, truth_data, noalloc=True)
        for k in KEYS:
            assert np.array_equal(a[0][k], b[0][k]), (n, k)
        assert np.array_equal(a[1], b[1]), n
        assert np.array_equal(a[2], b[2]), n
        assert a[2][1].sum() > 0 and a[2][0, 7] > 0 and a[2][0, 0] > 0


def test_noalloc_limits(B, truth_data):
    """The context without workspace refuses rjsmc_mutate; the allocation-free entry point
    refuses more particles than its static scratch holds, before launching anything."""
    bare = B.Context(W.system(), precision="f64", max_particles=0)
    n = 64
    p = B.empty_device_population(n, KC, KM)
    bare.init_prior(p, PR, 1)
    y = torch.as_tensor(truth_data, device="cuda")
    ll = bare.loglik(p, y)
    F = torch.zeros((1, M, D, D), dtype=torch.float64, device="cuda")
    kw = dict(seed=1, step=1, n_moves=1, n_sound=1, prior=PR, move_prob=(1, 1, 1, 1, 1, 1, 1, 0), z_move_sd=15.0,
              rw_scale=2.38, factors=F)
    g = torch.ones(1, dtype=torch.float64, device="cuda")
    with pytest.raises(B.RJSMCError) as e:
        bare.mutate(p, ll, B.empty_device_population(n, KC, KM), torch.empty_like(ll), g, None, y, None, **kw)
    assert e.value.status == B.RJSMC_E_INVALID and "max_particles" in str(e.value)
    big = B.RJSMC_NOALLOC_MAX_PARTICLES + 1
    import ctypes
    ps = B.particles_struct(p)
    ps.n = big
    ps.stride = big
    a = B.MutateArgs()
    a.seed, a.step, a.n_moves, a.n_sound = 1, 1, 1, 1
    for t in range(8):
        a.move_prob[t] = float(kw["move_prob"][t])
    a.z_move_sd, a.rw_scale = 15.0, 2.38
    a.factors = B._ptr(F)
    a.prior = B.make_prior(PR)
    st = B.lib().rjsmc_mutate_noalloc(bare._ptr, ctypes.byref(a), ctypes.byref(ps), B._ptr(ll), ctypes.byref(ps),
                                      B._ptr(ll), B._ptr(g), None, B._ptr(y), None, None, None, None)
    assert st == B.RJSMC_E_INVALID
    assert "RJSMC_NOALLOC_MAX_PARTICLES" in B.lib().rjsmc_last_error().decode()
