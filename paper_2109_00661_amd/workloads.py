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


def take(p, idx):
    """Sub-population with the particles at positions idx (a copy)."""
    idx = np.asarray(idx)
    out = dict(layout=p["layout"])
    for k, v in p.items():
        if k == "layout":
            continue
        out[k] = np.ascontiguousarray(v[..., idx])
    return out
