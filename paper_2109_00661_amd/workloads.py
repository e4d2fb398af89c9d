"""Seeded synthetic inputs: system description, prior-shaped particle populations, data noise.

This module holds no forward-model, likelihood or SMC arithmetic.  It only fixes the
acquisition system and draws seeded random inputs with the shapes and value ranges of
the paper's workloads (Section 4.1 synthetic study; priors of Section 2.3.1 with the
bounds of the synthetic configuration).  Both the HIP path and the CPU checks consume
these inputs; nothing here depends on either of them.

Particle populations are dicts of numpy arrays in structure-of-arrays form, particle
index fastest:

    kappa   int32[n]      conductivity interfaces (decoupled) or L-1 (merged)
    lambda  int32[n]      chargeability interfaces (decoupled; zero for merged)
    phi_b   f64[n]        log10 sigma_inf of the top segment
    phi     f64[KC, n]    log10 sigma_inf below each conductivity interface
    z_cond  f64[KC, n]    conductivity interface depths (m), ascending
    m       f64[KM, n]    chargeability below each chargeability interface (decoupled),
                          or per-layer chargeability, KC+1 rows (merged)
    z_charg f64[KM, n]    chargeability interface depths (m), ascending
    log10_tau, c  f64[n]  Cole-Cole time constant (log10 s) and frequency exponent
Slots beyond a particle's count are zero and are never read.
"""
import os
import numpy as np

LAYOUT_DECOUPLED = 0
LAYOUT_MERGED = 1

# Central-loop geometry and source (loop radius, height, current).
LOOP_RADIUS_M = 12.5
HEIGHT_M = 30.0
CURRENT_A = 1.0
N_FREQ = 40
N_GATE = 20
EPS_MN = 0.03            # multiplicative noise fraction
EPS_AN = 0.1             # additive noise floor, pT/s at 1 A, every gate

# Prior bounds of the synthetic configuration.
PRIOR = dict(kmax_cond=4, kmax_charg=3, phi_lo=-3.0, phi_hi=0.0, z_max=300.0,
             m_lo=0.0, m_hi=0.9, ltau_lo=-6.0, ltau_hi=-1.0, c_lo=0.1, c_hi=1.0)

_DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


def frequencies_hz():
    """40 frequencies log-spaced over 1 Hz .. 1 MHz."""
    return 10.0 ** (6.0 * np.arange(N_FREQ) / (N_FREQ - 1))


def gate_edges_s():
    """20 contiguous boxcar gates with log-spaced centres over 1e-5 .. 1e-2 s."""
    centres = 10.0 ** (-5.0 + 3.0 * np.arange(N_GATE) / (N_GATE - 1))
    half = 10.0 ** (1.5 / (N_GATE - 1))
    return centres / half, centres * half


def hankel_table():
    """(b_k, w_k) of the 120-point J1 filter stored beside this package."""
    t = np.loadtxt(os.path.join(_DATA, "hankel_j1_120.txt"))
    return np.ascontiguousarray(t[:, 0]), np.ascontiguousarray(t[:, 1])


def system(kmax_cond=PRIOR["kmax_cond"], kmax_charg=PRIOR["kmax_charg"]):
    b, w = hankel_table()
    lo, hi = gate_edges_s()
    return dict(loop_radius_m=LOOP_RADIUS_M, height_m=HEIGHT_M, current_a=CURRENT_A,
                freq_hz=frequencies_hz(), hankel_b=b, hankel_w=w,
                gate_open_s=lo, gate_close_s=hi, eps_mn=EPS_MN,
                eps_an=np.full(N_GATE, EPS_AN), kmax_cond=kmax_cond, kmax_charg=kmax_charg,
                z_max_m=PRIOR["z_max"])


def empty_particles(n, kc, km, layout=LAYOUT_DECOUPLED):
    rows_m = kc + 1 if layout == LAYOUT_MERGED else km
    return dict(layout=layout, kappa=np.zeros(n, np.int32), lambda_=np.zeros(n, np.int32),
                phi_b=np.zeros(n), phi=np.zeros((kc, n)), z_cond=np.zeros((kc, n)),
                m=np.zeros((rows_m, n)), z_charg=np.zeros((km, n)),
                log10_tau=np.zeros(n), c=np.zeros(n))


def truth_three_layer():
    """Three-layer truth of the synthetic study: 0.01 / 0.1 / 0.001 S/m, interfaces at
    20 m and 40 m, the middle layer chargeable (m=0.4, tau=1e-3 s, c=0.5).  Decoupled
    encoding: two conductivity interfaces, two chargeability interfaces (the second one
    returns to m=0)."""
    p = empty_particles(1, PRIOR["kmax_cond"], PRIOR["kmax_charg"])
    p["kappa"][0] = 2
    p["phi_b"][0] = -2.0
    p["phi"][:2, 0] = [-1.0, -3.0]
    p["z_cond"][:2, 0] = [20.0, 40.0]
    p["lambda_"][0] = 2
    p["m"][:2, 0] = [0.4, 0.0]
    p["z_charg"][:2, 0] = [20.0, 40.0]
    p["log10_tau"][0] = -3.0
    p["c"][0] = 0.5
    return p


def truth_three_layer_merged():
    """The same three-layer truth in the merged layout (three layers, per-layer m)."""
    p = empty_particles(1, 2, 0, LAYOUT_MERGED)
    p["kappa"][0] = 2
    p["phi_b"][0] = -2.0
    p["phi"][:, 0] = [-1.0, -3.0]
    p["z_cond"][:, 0] = [20.0, 40.0]
    p["m"][:, 0] = [0.0, 0.4, 0.0]
    p["log10_tau"][0] = -3.0
    p["c"][0] = 0.5
    return p


def near_truth_merged(n, seed=0, kc=4):
    """Merged-layout particles near the three-layer truth (stand-ins for posterior
    samples near the mode): particle 0 is the truth itself, the others perturb it by
    Gaussian draws of sd 0.02 in each log10 sigma, 0.5 m in each interface depth, 0.01
    in the middle layer's m, 0.02 in log10 tau and 0.01 in c.  Capacity kc >= 2 rows
    (only three layers are used)."""
    rng = np.random.default_rng(seed)
    p = empty_particles(n, kc, 0, LAYOUT_MERGED)
    jitter = lambda sd, *shape: sd * rng.standard_normal(shape) * (np.arange(n) > 0)
    p["kappa"][:] = 2
    p["phi_b"][:] = -2.0 + jitter(0.02, n)
    p["phi"][:2] = np.array([[-1.0], [-3.0]]) + jitter(0.02, 2, n)
    p["z_cond"][:2] = np.array([[20.0], [40.0]]) + jitter(0.5, 2, n)
    p["m"][1] = 0.4 + jitter(0.01, n)
    p["log10_tau"][:] = -3.0 + jitter(0.02, n)
    p["c"][:] = 0.5 + jitter(0.01, n)
    return p


def data_noise(seed=1):
    """Standard-normal draws that scale the data noise of the synthetic sounding."""
    return np.random.default_rng(seed).standard_normal(N_GATE)


def merged_population(n, n_layers=5, seed=2, kc=None):
    """Merged-layout particles, each an n_layers Cole-Cole model drawn from the prior
    ranges: interfaces sorted U(0, z_max), log10 sigma ~ U[-3,0] and m ~ U[0,0.9] per
    layer, log10 tau ~ U[-6,-1], c ~ U[0.1,1]."""
    kc = n_layers - 1 if kc is None else kc
    rng = np.random.default_rng(seed)
    p = empty_particles(n, kc, 0, LAYOUT_MERGED)
    P = PRIOR
    p["kappa"][:] = n_layers - 1
    p["z_cond"][:n_layers - 1] = np.sort(rng.uniform(0.0, P["z_max"], (n_layers - 1, n)), axis=0)
    sig = rng.uniform(P["phi_lo"], P["phi_hi"], (n_layers, n))
    p["phi_b"][:] = sig[0]
    p["phi"][:n_layers - 1] = sig[1:]
    p["m"][:n_layers] = rng.uniform(P["m_lo"], P["m_hi"], (n_layers, n))
    p["log10_tau"][:] = rng.uniform(P["ltau_lo"], P["ltau_hi"], n)
    p["c"][:] = rng.uniform(P["c_lo"], P["c_hi"], n)
    return p


def decoupled_population(n, kmax_cond, kmax_charg, seed=3, min_sep=0.0, kappa=None, lam=None):
    """Decoupled-layout particles drawn from the prior: kappa ~ U{0..kmax_cond},
    lambda ~ U{0..kmax_charg} (or fixed), parameters from the prior ranges.  With
    min_sep > 0 the draw is repeated for any particle whose interfaces (over both
    partitions) come closer than min_sep metres or closer than min_sep to the surface."""
    rng = np.random.default_rng(seed)
    P = PRIOR
    p = empty_particles(n, kmax_cond, kmax_charg)
    p["kappa"][:] = rng.integers(0, kmax_cond + 1, n) if kappa is None else kappa
    p["lambda_"][:] = rng.integers(0, kmax_charg + 1, n) if lam is None else lam
    p["phi_b"][:] = rng.uniform(P["phi_lo"], P["phi_hi"], n)
    p["log10_tau"][:] = rng.uniform(P["ltau_lo"], P["ltau_hi"], n)
    p["c"][:] = rng.uniform(P["c_lo"], P["c_hi"], n)
    for i in range(n):
        k, l = int(p["kappa"][i]), int(p["lambda_"][i])
        while True:
            zc = np.sort(rng.uniform(0.0, P["z_max"], k))
            zm = np.sort(rng.uniform(0.0, P["z_max"], l))
            allz = np.sort(np.concatenate([[0.0], zc, zm]))
            if min_sep <= 0.0 or np.all(np.diff(allz) >= min_sep):
                break
        p["z_cond"][:k, i] = zc
        p["z_charg"][:l, i] = zm
        p["phi"][:k, i] = rng.uniform(P["phi_lo"], P["phi_hi"], k)
        p["m"][:l, i] = rng.uniform(P["m_lo"], P["m_hi"], l)
    return p


def prior_population(n, kmax_cond, kmax_charg, seed=3, n_per_sounding=0):
    """Decoupled-layout particles from the prior drawn in bulk (vectorised; large
    batches): kappa ~ U{0..kmax_cond}, lambda ~ U{0..kmax_charg}, sorted U(0, z_max)
    interfaces in the used rows (zeros beyond), properties from the prior ranges."""
    rng = np.random.default_rng(seed)
    P = PRIOR
    p = empty_particles(n, kmax_cond, kmax_charg)
    p["n_per_sounding"] = n_per_sounding
    p["kappa"][:] = rng.integers(0, kmax_cond + 1, n)
    p["lambda_"][:] = rng.integers(0, kmax_charg + 1, n)
    p["phi_b"][:] = rng.uniform(P["phi_lo"], P["phi_hi"], n)
    p["log10_tau"][:] = rng.uniform(P["ltau_lo"], P["ltau_hi"], n)
    p["c"][:] = rng.uniform(P["c_lo"], P["c_hi"], n)
    for key, kmax, cnt in (("z_cond", kmax_cond, p["kappa"]), ("z_charg", kmax_charg, p["lambda_"])):
        if kmax == 0:
            continue
        z = rng.uniform(0.0, P["z_max"], (kmax, n))
        rows = np.arange(kmax)[:, None]
        z = np.where(rows < cnt[None, :], z, np.inf)
        z = np.sort(z, axis=0)
        p[key][:] = np.where(np.isfinite(z), z, 0.0)
    if kmax_cond:
        p["phi"][:] = rng.uniform(P["phi_lo"], P["phi_hi"], (kmax_cond, n))
    if kmax_charg:
        p["m"][:] = rng.uniform(P["m_lo"], P["m_hi"], (kmax_charg, n))
    return p


def survey(n_lines=10, n_stations=200, station_m=25.0, line_m=100.0):
    """Synthetic airborne survey standing in for a flight-line dataset: n_lines parallel
    lines of n_stations soundings.  Every station's truth is a three-layer model with
    smoothly varying conductivities and interface depths; an elliptical chargeable body
    (about 40% of the stations of the default grid) makes the second layer chargeable with
    m up to 0.6 (tapering to the body's edge), tau from 1e-4 s to 1e-2 s across it and
    c = 0.5.  Returns (truth particles in the decoupled layout with capacities
    kmax_cond = 4, kmax_charg = 3, body mask [S], x [S], y [S])."""
    x = np.tile(np.arange(n_stations) * station_m, n_lines)
    y = np.repeat(np.arange(n_lines) * line_m, n_stations)
    S = n_lines * n_stations
    xs, ys = x.max() if S > 1 else 1.0, y.max() if n_lines > 1 else 1.0
    two_pi = 2.0 * np.pi
    phi1 = -2.0 + 0.3 * np.sin(two_pi * x / 2000.0) + 0.2 * np.cos(two_pi * y / 700.0)
    phi2 = -1.0 + 0.3 * np.cos(two_pi * x / 1300.0)
    phi3 = -2.5 + 0.3 * np.sin(two_pi * y / 900.0)
    z1 = 20.0 + 10.0 * np.sin(two_pi * (x + y) / 1500.0)
    z2 = z1 + 20.0
    cx, cy = 0.5 * xs, 0.5 * ys
    ax, ay = 0.30 * xs, 0.50 * max(ys, 1.0)
    r2 = ((x - cx) / ax) ** 2 + ((y - cy) / ay) ** 2
    body = r2 < 1.0
    p = empty_particles(S, PRIOR["kmax_cond"], PRIOR["kmax_charg"])
    p["kappa"][:] = 2
    p["phi_b"][:] = phi1
    p["phi"][0] = phi2
    p["phi"][1] = phi3
    p["z_cond"][0] = z1
    p["z_cond"][1] = z2
    p["lambda_"][:] = np.where(body, 2, 0)
    p["z_charg"][0] = np.where(body, z1, 0.0)
    p["z_charg"][1] = np.where(body, z2, 0.0)
    p["m"][0] = np.where(body, 0.6 * np.sqrt(np.clip(1.0 - r2, 0.0, 1.0)), 0.0)
    p["log10_tau"][:] = -4.0 + 2.0 * np.clip((x - (cx - ax)) / (2.0 * ax), 0.0, 1.0)
    p["c"][:] = 0.5
    return p, body, x, y


def take(p, idx):
    """Sub-population with the particles at positions idx (a copy)."""
    idx = np.asarray(idx)
    out = dict(layout=p["layout"])
    for k, v in p.items():
        if k == "layout":
            continue
        out[k] = np.ascontiguousarray(v[..., idx])
    return out
