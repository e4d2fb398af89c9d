"""Pins of the oracle forward model against what mathematics and the paper fix.

Each test checks the oracle against something other than itself: closed forms,
textbook special cases, an algebraically different formulation at high precision,
adaptive quadrature of the defining integral, or invariants.
"""
import numpy as np
import mpmath as mp
import pytest
from scipy.integrate import quad
from scipy.special import j1, sici, erf

from oracle import em
from paper_2109_00661_amd import workloads as W

MU0 = 4e-7 * np.pi


# ---------------------------------------------------------------- Cole-Cole (Section 2)
def test_cole_cole_limits():
    w = 2 * np.pi * np.array([1.0, 1e3, 1e6])
    s = 0.05
    # m = 0: conductive-only model, exactly sigma_inf
    assert np.all(em.cole_cole(s, 0.0, 1e-3, 0.5, w) == s)
    # tau -> 0: the dispersion term -> 1, sigma_hat -> sigma_inf (1 - m) = sigma_s
    np.testing.assert_allclose(em.cole_cole(s, 0.3, 1e-30, 0.7, w), s * 0.7, rtol=1e-12)
    # tau -> inf: sigma_hat -> sigma_inf
    np.testing.assert_allclose(em.cole_cole(s, 0.3, 1e30, 0.7, w), s, rtol=1e-12)
    # c = 1 is the Debye relaxation
    tau = 2e-4
    np.testing.assert_allclose(em.cole_cole(s, 0.3, tau, 1.0, w), s - s * 0.3 / complex(1.0, 0.0) / (1 + 1j * w * tau),
                               rtol=1e-14)
    # c = 1/2: (i w tau)^(1/2) = sqrt(w tau) (1+i)/sqrt(2)
    z = np.sqrt(w * tau) * (1 + 1j) / np.sqrt(2)
    np.testing.assert_allclose(em.cole_cole(s, 0.3, tau, 0.5, w), s * (1 - 0.3 / (1 + z)), rtol=1e-14)


def test_cole_cole_chargeability_definition():
    """m = (sigma_inf - sigma_s)/sigma_inf: the DC limit equals sigma_s."""
    s_inf, s_s = 0.2, 0.15
    m = (s_inf - s_s) / s_inf
    np.testing.assert_allclose(em.cole_cole(s_inf, m, 1.0, 0.6, 1e-30), s_s, rtol=1e-12)


# ------------------------------------------------------- TE reflection (Ward & Hohmann)
def _rte_admittance_mp(lam, w, sig_hat, thick, dps=40):
    """Admittance form of the layered-earth TE reflection at high precision:
    U_N = u_N; U_l = u_l (U_{l+1} + u_l tanh(u_l h_l)) / (u_l + U_{l+1} tanh(u_l h_l));
    r = (lam - U_0) / (lam + U_0)."""
    with mp.workdps(dps):
        mu0 = 4 * mp.pi * mp.mpf(10) ** -7
        lam = mp.mpf(lam)
        u = [mp.sqrt(lam ** 2 + 1j * mp.mpf(w) * mu0 * mp.mpc(s)) for s in sig_hat]
        U = u[-1]
        for l in range(len(sig_hat) - 2, -1, -1):
            t = mp.tanh(u[l] * mp.mpf(thick[l]))
            U = u[l] * (U + u[l] * t) / (u[l] + U * t)
        return complex((lam - U) / (lam + U))


@pytest.mark.parametrize("f", [1.0, 1e2, 1e4, 1e6])
@pytest.mark.parametrize("lam", [1e-4, 3e-3, 0.05, 0.4])
def test_reflection_matches_admittance_form(f, lam):
    w = 2 * np.pi * f
    sig_hat = [em.cole_cole(0.01, 0.0, 1e-3, 0.5, w), em.cole_cole(0.1, 0.4, 1e-3, 0.5, w),
               em.cole_cole(0.001, 0.0, 1e-3, 0.5, w), em.cole_cole(0.3, 0.7, 1e-2, 0.3, w)]
    thick = [20.0, 20.0, 55.0]
    k2 = [1j * w * MU0 * s for s in sig_hat]
    r = em.reflection_te(np.array(lam), k2, thick)
    ref = _rte_admittance_mp(lam, w, sig_hat, thick)
    assert abs(r - ref) <= 1e-12 * abs(ref)


def test_reflection_halfspace_textbook():
    lam = np.logspace(-5, 0.5, 40)
    w = 2 * np.pi * 1e3
    k2 = 1j * w * MU0 * 0.02
    u = np.sqrt(lam ** 2 + k2)
    np.testing.assert_allclose(em.reflection_te(lam, [k2], []), (lam - u) / (lam + u), rtol=1e-9)


def test_identical_layers_collapse_to_halfspace_bitexact():
    lam = np.logspace(-5, 0.5, 60)[None, :]
    w = 2 * np.pi * np.logspace(0, 6, 7)[:, None]
    k2 = 1j * w * MU0 * em.cole_cole(0.03, 0.35, 1e-3, 0.6, w)
    r3 = em.reflection_te(lam, [k2, k2, k2], [17.0, 44.0])
    r1 = em.reflection_te(lam, [k2], [])
    assert np.array_equal(r3, r1)


def test_zero_thickness_layer_is_transparent():
    lam = np.logspace(-5, 0.5, 60)[None, :]
    w = 2 * np.pi * np.logspace(0, 6, 7)[:, None]
    ka = 1j * w * MU0 * 0.01
    kb = 1j * w * MU0 * em.cole_cole(0.5, 0.6, 1e-4, 0.4, w)
    kc = 1j * w * MU0 * 0.002
    with_zero = em.reflection_te(lam, [ka, kb, kc], [25.0, 0.0])
    without = em.reflection_te(lam, [ka, kc], [25.0])
    np.testing.assert_allclose(with_zero, without, rtol=1e-12, atol=0)


def test_low_frequency_born_limit():
    """At low induction number r_TE ~ -(i w mu0 / (2 lam)) int sigma(z) exp(-2 lam z) dz."""
    w = 2 * np.pi * 1e-3
    lam = 0.05
    sig = [0.01, 0.1, 0.001]
    z = [0.0, 20.0, 40.0]
    born = 0.0
    for l, s in enumerate(sig):
        bot = np.exp(-2 * lam * z[l + 1]) if l + 1 < len(z) else 0.0
        born += s * (np.exp(-2 * lam * z[l]) - bot) / (2 * lam)
    born *= -1j * w * MU0 / (2 * lam)
    r = em.reflection_te(np.array(lam), [1j * w * MU0 * s for s in sig], [20.0, 20.0])
    assert abs(r - born) <= 1e-6 * abs(born)


# ------------------------------------------------------------- J1 Hankel filter (O-5)
@pytest.mark.parametrize("r", [1e-4, 1e-3, 1e-2, 0.1, 0.5, 1.0])
def test_filter_closed_form_pairs(r):
    b, wt = W.hankel_table()
    lam = b / r
    pairs = [
        (lam * np.exp(-lam), r / (1 + r * r) ** 1.5),
        (np.exp(-lam), (np.sqrt(1 + r * r) - 1) / (r * np.sqrt(1 + r * r))),
        (np.exp(-lam) / lam, (np.sqrt(1 + r * r) - 1) / r),
    ]
    for f, F in pairs:
        assert abs(np.sum(wt * f) / r - F) <= 2e-5 * abs(F)


def test_filter_gaussian_pair():
    b, wt = W.hankel_table()
    for r in [0.05, 0.3, 1.0, 1.8]:
        lam = b / r
        F = r / 4 * np.exp(-r * r / 4)
        assert abs(np.sum(wt * lam ** 2 * np.exp(-lam ** 2)) / r - F) <= 2e-5 * F


def _hz_quadrature(system, sig, ms, thick, tau, c, f):
    """(I a / 2) int_0^inf r_TE e^{-2 lam h} lam J1(lam a) dlam by adaptive quadrature."""
    a, h, I = system["loop_radius_m"], system["height_m"], system["current_a"]
    w = 2 * np.pi * f
    k2 = [1j * w * MU0 * em.cole_cole(s, m, tau, c, w) for s, m in zip(sig, ms)]

    def integrand(L, part):
        v = em.reflection_te(np.array(L), k2, thick) * np.exp(-2 * L * h) * L * j1(L * a)
        return v.real if part == 0 else v.imag

    edges = np.concatenate([[0.0], np.logspace(-8, 0.3, 70)])
    out = 0j
    for part in (0, 1):
        tot = sum(quad(integrand, edges[i], edges[i + 1], args=(part,), epsabs=0, epsrel=1e-12,
                       limit=200)[0] for i in range(len(edges) - 1))
        out += tot if part == 0 else 1j * tot
    return I * a / 2 * out


@pytest.mark.parametrize("model", ["half1e-3", "half1", "truth"])
def test_secondary_field_against_quadrature(system, model):
    if model == "half1e-3":
        sig, ms, thick, tau, c = [1e-3], [0.0], [], 1e-3, 0.5
    elif model == "half1":
        sig, ms, thick, tau, c = [1.0], [0.0], [], 1e-3, 0.5
    else:
        sig, ms, thick, tau, c = [0.01, 0.1, 0.001], [0.0, 0.4, 0.0], [20.0, 20.0], 1e-3, 0.5
    H = em.secondary_hz(system, sig, ms, thick, tau, c)
    for j in [0, 7, 13, 20, 26, 33, 39]:
        ref = _hz_quadrature(system, sig, ms, thick, tau, c, system["freq_hz"][j])
        assert abs(H[j] - ref) <= 1e-5 * abs(ref), (j, H[j], ref)


def test_secondary_field_perfect_conductor_image(system):
    """r_TE -> -1: the image of the loop, H^s = -I a^2 / (2 (a^2 + 4 h^2)^(3/2))."""
    a, h = system["loop_radius_m"], system["height_m"]
    H = em.secondary_hz(system, [1e6], [0.0], [], 1e-3, 0.5)
    img = -a * a / (2 * (a * a + 4 * h * h) ** 1.5)
    assert abs(H[-1].real - img) <= 1e-3 * abs(img)


# ----------------------------------------------------- frequency-to-time transform (O-6)
def test_time_kernel_constant_spectrum_is_zero(system, K_oracle):
    """Constant Im H / w transforms to a delta at t = 0, so every off-time gate is 0."""
    w = 2 * np.pi * system["freq_hz"]
    y = K_oracle @ w
    scale = np.abs(K_oracle * w[None, :]).sum(axis=1)
    assert np.all(np.abs(y) <= 1e-10 * scale)


def test_time_kernel_linear_spectrum_sine_integral(system, K_oracle):
    """Im H / w = alpha + beta ln w (reproduced exactly by the natural spline) has
    F(t) = beta [Si(w_1 t) - Si(w_n t)] / t in closed form."""
    w = 2 * np.pi * system["freq_hz"]
    alpha, beta = 0.7, -0.3
    G = w * (alpha + beta * np.log(w))
    lo, hi = system["gate_open_s"], system["gate_close_s"]

    def F(t):
        return beta * (sici(w[0] * t)[0] - sici(w[-1] * t)[0]) / t

    ref = -(2 / np.pi) * MU0 * 1e12 * (F(lo) - F(hi)) / (hi - lo)
    y = K_oracle @ G
    scale = np.abs(K_oracle * G[None, :]).sum(axis=1)
    # the late-gate entries of high-frequency columns are small differences of large
    # oscillatory moments; QUADPACK reaches ~1e-11 of the row scale there
    assert np.all(np.abs(y - ref) <= 1e-10 * scale)


@pytest.mark.parametrize("m,pw,t", [(0, 0, 1e-5), (0, 3, 1.2e-2), (12, 2, 3e-4), (25, 1, 1e-3),
                                     (30, 3, 3e-5), (38, 2, 1.2e-2), (38, 3, 2e-3)])
def test_time_kernel_cos_moments_brute_force(system, m, pw, t):
    """The oscillatory moments int_{w_m}^{w_m+1} (ln w - ln w_m)^p cos(w t) dw against
    Gauss-Legendre panels of at most a quarter period each (a different rule)."""
    w = 2 * np.pi * system["freq_hz"]
    got = em.cos_moments(system["freq_hz"], np.array([t]))[m, pw, 0]
    npan = int(np.ceil((w[m + 1] - w[m]) * t / (np.pi / 2))) + 1
    edges = np.linspace(w[m], w[m + 1], npan + 1)
    xg, wg = np.polynomial.legendre.leggauss(24)
    mid = 0.5 * (edges[1:] + edges[:-1])[:, None]
    half = 0.5 * (edges[1:] - edges[:-1])[:, None]
    om = mid + half * xg[None, :]
    vals = (np.log(om) - np.log(w[m])) ** pw * np.cos(om * t)
    ref = np.sum(math_fsum_rows(vals * wg[None, :] * half))
    scale = np.sum(np.abs(vals * wg[None, :] * half))
    assert abs(got - ref) <= 1e-13 * scale + 1e-13 * abs(ref), (got, ref, scale)


def math_fsum_rows(a):
    import math
    return np.array([math.fsum(r) for r in a])


def _halfspace_hz_closed_form(w, s, a):
    """Ward & Hohmann: total H_z at the centre of a loop on a half-space (h = 0),
    minus the free-space primary I/(2a); computed at 40 digits."""
    with mp.workdps(40):
        k = mp.sqrt(-1j * mp.mpf(w) * 4 * mp.pi * mp.mpf(10) ** -7 * mp.mpf(s))
        if mp.im(k) > 0:
            k = -k
        a = mp.mpf(a)
        Ht = -1 / (k ** 2 * a ** 3) * (3 - (3 + 3j * k * a - k ** 2 * a ** 2) * mp.exp(-1j * k * a))
        return complex(Ht - 1 / (2 * a))


def _halfspace_gate_closed_form(t_lo, t_hi, s, a):
    """Step-off -dBz/dt averaged over a gate: mu0 [h_z(t_lo) - h_z(t_hi)] / (t_hi - t_lo)
    with h_z(t) = (I/2a)[3 e^{-x^2}/(sqrt(pi) x) + (1 - 3/(2x^2)) erf(x)], x = a sqrt(mu0 s/4t)."""
    def hz(t):
        x = a * np.sqrt(MU0 * s / (4 * t))
        return 1 / (2 * a) * (3 * np.exp(-x * x) / (np.sqrt(np.pi) * x) + (1 - 3 / (2 * x * x)) * erf(x))
    return MU0 * 1e12 * (hz(t_lo) - hz(t_hi)) / (t_hi - t_lo)


@pytest.mark.parametrize("s,med_tol,max_tol", [(1.0, 1e-4, 2e-3), (0.1, 1e-4, 2e-3), (0.01, 1e-2, 0.1)])
def test_time_domain_halfspace_closed_form(system, K_oracle, s, med_tol, max_tol):
    a = system["loop_radius_m"]
    w = 2 * np.pi * system["freq_hz"]
    G = np.array([_halfspace_hz_closed_form(wi, s, a).imag for wi in w])
    y = K_oracle @ G
    ref = _halfspace_gate_closed_form(system["gate_open_s"], system["gate_close_s"], s, a)
    rel = np.abs(y - ref) / np.abs(ref)
    assert np.median(rel) < med_tol and rel.max() < max_tol, rel


# -------------------------------------------------------------- likelihood (Section 2.3.2)
def test_loglik_at_exact_fit_and_textbook_gaussian(system):
    from scipy.stats import norm
    rng = np.random.default_rng(5)
    y = rng.normal(0, 100, 20)
    ll = em.loglik_from_response(y, y, system["eps_an"], system["eps_mn"])
    s2 = system["eps_an"] ** 2 + (system["eps_mn"] * y) ** 2
    assert abs(ll - (-0.5 * np.sum(np.log(2 * np.pi * s2)))) <= 1e-12 * abs(ll)
    d = y + rng.normal(0, 1, 20)
    ll0 = em.loglik_from_response(y, d, system["eps_an"], 0.0)
    ref = np.sum(norm.logpdf(d, loc=y, scale=system["eps_an"]))
    assert abs(ll0 - ref) <= 1e-12 * abs(ref)


# ---------------------------------------------------------------- qualitative (Section 2)
def test_conductive_only_positive_and_ip_sign_reversal(system, K_oracle):
    p = W.truth_three_layer()
    y_ip = em.forward(p, system, K_oracle)[0]
    p0 = W.truth_three_layer()
    p0["m"][:] = 0.0
    y_c = em.forward(p0, system, K_oracle)[0]
    assert np.all(y_c > 0)                # conductive-only data are positive
    assert y_ip.min() < 0                 # chargeable layer produces negative late-time data
    assert np.all(np.diff(y_c) < 0)       # monotone decay


def test_merged_and_decoupled_layouts_agree(system, K_oracle):
    """A decoupled particle and its merged equivalent give the same response."""
    d = W.truth_three_layer()
    mg = W.truth_three_layer_merged()
    np.testing.assert_allclose(em.forward(mg, system, K_oracle), em.forward(d, system, K_oracle), rtol=1e-12)


# --------------------------------------------------------------------- gradient (O-8)
def _fd_grad(p, system, K, d, i, name, row, rel=1e-6):
    x0 = p[name][i] if row is None else p[name][row, i]
    hstep = rel * max(abs(x0), 1.0)
    vals = []
    for sgn in (1, -1):
        q = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in p.items()}
        if row is None:
            q[name][i] = x0 + sgn * hstep
        else:
            q[name][row, i] = x0 + sgn * hstep
        vals.append(em.loglik(q, system, K, d, [i])[0])
    return (vals[0] - vals[1]) / (2 * hstep)


@pytest.mark.parametrize("layout", ["decoupled", "merged"])
def test_gradient_against_central_differences(system, K_oracle, truth_data, layout):
    if layout == "decoupled":
        p = W.decoupled_population(3, 3, 2, seed=11, min_sep=2.0, kappa=np.array([3, 1, 2]),
                                   lam=np.array([2, 1, 0]))
    else:
        p = W.merged_population(2, 4, seed=12)
    ll, g = em.loglik_grad(p, system, K_oracle, truth_data)
    np.testing.assert_allclose(ll, em.loglik(p, system, K_oracle, truth_data), rtol=1e-12)
    for i in range(len(p["kappa"])):
        names = em.particle_params(p, i)
        gvec = np.array([g[n][i] if r is None else g[n][r, i] for n, r in names])
        fd = np.array([_fd_grad(p, system, K_oracle, truth_data, i, n, r) for n, r in names])
        assert np.max(np.abs(gvec - fd)) <= 1e-6 * np.max(np.abs(gvec)), (i, gvec, fd)


def test_gradient_structural_zeros(system, K_oracle, truth_data):
    # no chargeable segment: tau and c do not enter the response
    p = W.decoupled_population(2, 3, 2, seed=13, kappa=np.array([2, 1]), lam=np.array([0, 0]))
    _, g = em.loglik_grad(p, system, K_oracle, truth_data)
    assert np.all(g["log10_tau"] == 0) and np.all(g["c"] == 0)
    # an interface between two identical conductivities has zero depth derivative
    p = W.decoupled_population(1, 3, 0, seed=14, kappa=np.array([2]), lam=np.array([0]))
    p["phi"][0, 0] = p["phi_b"][0]
    _, g = em.loglik_grad(p, system, K_oracle, truth_data)
    gmax = max(abs(g["phi_b"][0]), np.abs(g["phi"][:, 0]).max())
    assert abs(g["z_cond"][0, 0]) <= 1e-12 * gmax and abs(g["z_cond"][1, 0]) > 1e-6 * gmax
