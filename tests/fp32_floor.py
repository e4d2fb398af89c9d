"""Rounding floor of the FP32 forward variant (test helper, oracle arithmetic only).

The FP32 variant runs the layer recursion in FP32 and accumulates the Hankel sum, the
time transform and the likelihood in FP64.  The most it can deliver for a reflection
term is Im r_TE correctly rounded to float32; this helper evaluates the oracle's FP64
terms, rounds each to float32 and carries both through the FP64 filter sum and time
transform, so that the response and log-likelihood differences are the floor any FP32
recursion incurs."""
import numpy as np

from oracle import em


def reflection_terms(system, p, i):
    """(c_k [nh], Im r_TE [nf, nh]) of particle i by the oracle (Section 2 forward model)."""
    sig, ms, thick = em.merged_stack(p, i)
    a, h = system["loop_radius_m"], system["height_m"]
    w = 2.0 * np.pi * np.asarray(system["freq_hz"])[:, None]
    lam = (np.asarray(system["hankel_b"]) / a)[None, :]
    ck = 0.5 * system["current_a"] * np.asarray(system["hankel_w"]) * lam[0] * np.exp(-2.0 * lam[0] * h)
    tau = 10.0 ** p["log10_tau"][i]
    k2 = [1j * w * em.MU0 * em.cole_cole(sig[l], ms[l], tau, p["c"][i], w) for l in range(len(sig))]
    return ck, em.reflection_te(lam, k2, thick).imag


def floor(system, K, p, i, d):
    """For particle i: oracle response y, the response y32 of float32-rounded terms,
    A_g = sum_j |K_gj| sum_k |c_k Im r| and the two log-likelihoods (ll, ll32)."""
    ck, im = reflection_terms(system, p, i)
    y = K @ (im @ ck)
    y32 = K @ (im.astype(np.float32).astype(np.float64) @ ck)
    A = np.abs(K) @ (np.abs(im) @ np.abs(ck))
    ll = em.loglik_from_response(y, d, system["eps_an"], system["eps_mn"])
    ll32 = em.loglik_from_response(y32, d, system["eps_an"], system["eps_mn"])
    return y, y32, A, ll, ll32
