"""Benchmark of the RJSMC hot path on one MI355X.

Headline: forward model + log-likelihood evaluations per second for 65,536 particles,
each a five-layer Cole-Cole model drawn from the prior ranges, with the 40-frequency /
120-point J1 / 20-gate central-loop system (FP64).  One step = one rjsmc_loglik launch
over the whole batch; inputs are resident in HBM before the timed region.

Prints one JSON line.  Options: --steps K --warmup W --gpus N (only 1 is supported)
--no-cpu (skip the CPU oracle baseline) --quick (skip the survey and the move comparison).
"""
import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2109_00661_amd import workloads as W  # noqa: E402

N_PARTICLES = 65536
N_LAYERS = 5
# Nominal floating-point work of one layer step of the reflection recursion (complex
# square root, interface term, propagation exponential, recursion update), counting
# each sqrt, division, exp and sincos as one operation; see the design notes.
FLOP_PER_LAYER_STEP = 66
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3
# Sources of the headline kernel, and the committed hardware-counter summary of its HBM
# traffic; the summary is used only while it was taken on these exact sources.
KERNEL_SOURCES = ("forward.hip", "recursion.h", "cplx.h", "merge.h", "rjsmc_internal.h")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "forward_kernel_65536x5layer_fp64_hbm_traffic.txt")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2109_00661_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per headline launch (FETCH_SIZE + WRITE_SIZE, calibrated against a copy
    of known size) from the committed counter summary, or None when the summary is
    missing or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_PROFILE) as f:
            fields = dict(line.split(":", 1) for line in f if re.match(r"^[a-z_0-9]+:", line))
    except OSError:
        return None
    if fields.get("sources_sha256", "").strip() != kernel_sources_sha256():
        return None
    return float(fields["hbm_bytes_per_launch"])


def nominal_flop_per_eval(n_layers, n_freq=40, n_hankel=120):
    return n_freq * n_hankel * n_layers * FLOP_PER_LAYER_STEP


def synth_response():
    """Gate responses of the three-layer truth (device forward model)."""
    from paper_2109_00661_amd import binding as B
    ctx = B.Context(W.system(kmax_cond=2, kmax_charg=0), precision="f64")
    y = ctx.forward(B.particles_to_device(W.truth_three_layer_merged())).cpu().numpy()[0]
    ctx.check()
    return y


def synth_data(torch):
    """Synthetic sounding: the three-layer truth through the forward model plus noise
    with the standard deviation of the noise model at the response."""
    system = W.system(kmax_cond=2, kmax_charg=0)
    y = synth_response()
    s = np.sqrt(system["eps_an"] ** 2 + (system["eps_mn"] * y) ** 2)
    return torch.as_tensor(y + s * W.data_noise(1), device="cuda")


def copy_calibration(torch, mib):
    """One plain device-to-device copy of `mib` MiB, whose FETCH_SIZE / WRITE_SIZE
    readings scale the counters of the kernels profiled in the same run."""
    if mib <= 0:
        return
    src = torch.ones((mib << 20) // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def time_calls(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        fn()
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(end) / steps, wall


# ------------------------------------------------------------------ CPU baseline (oracle)
_ORACLE = {}


def _oracle_setup():
    """The oracle's system, K and synthetic data (the three-layer truth through the
    oracle's forward model plus the seeded noise), computed once per process."""
    if not _ORACLE:
        import warnings
        from oracle import em
        system = W.system(kmax_cond=N_LAYERS - 1, kmax_charg=0)
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            K = em.make_K(system)
        y = em.forward(W.truth_three_layer_merged(), system, K)[0]
        d = y + np.sqrt(em.noise_variance(y, system["eps_an"], system["eps_mn"])) * W.data_noise(1)
        _ORACLE.update(system=system, K=K, d=d, pop=W.merged_population(N_PARTICLES, N_LAYERS, seed=2,
                                                                        kc=N_LAYERS - 1))
    return _ORACLE


def _oracle_chunk(bounds):
    """Forward + log-likelihood of particles [lo, hi) of the headline batch by the oracle."""
    from oracle import em
    o = _oracle_setup()
    lo, hi = bounds
    em.loglik(o["pop"], o["system"], o["K"], o["d"], range(lo, hi))
    return hi - lo


def cpu_host():
    """Host CPU model and the number of cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    share = int(os.environ.get("OMP_NUM_THREADS", avail) or avail)
    return model, avail, max(1, min(avail, share))


def cpu_baseline(budget_s=6.0, repeats=3):
    """The oracle as it stands, timed on the host: forward + log-likelihood evaluations of
    the headline batch's particles on one thread and on a process pool over the host's
    cores (median of `repeats` runs of about `budget_s` each, on consecutive particles of
    the same batch), and complete Algorithm-1 steps of one 256-particle sounding
    extrapolated to a whole run.  Run before the GPU is touched (the pool forks)."""
    import multiprocessing as mp
    model, avail, workers = cpu_host()
    _oracle_setup()
    chunk = 32
    one, start = [], 0
    for _ in range(repeats):
        n, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            n += _oracle_chunk((start + n, start + n + chunk))
        one.append(n / (time.perf_counter() - t0))
        start += n
    many = []
    with mp.get_context("fork").Pool(workers) as pool:
        pool.map(_oracle_chunk, [(0, 1)] * workers)            # warm the workers
        for _ in range(repeats):
            n_jobs = max(workers, int(np.median(one) * budget_s * workers * 0.9) // chunk)
            jobs = [((q * chunk) % N_PARTICLES, (q * chunk) % N_PARTICLES + chunk) for q in range(n_jobs)]
            t0 = time.perf_counter()
            n = sum(pool.map(_oracle_chunk, jobs, chunksize=1))
            many.append(n / (time.perf_counter() - t0))
    out = dict(value=float(np.median(many)), unit="evals/s", cores=workers, kind="oracle",
               sample="forward+loglik (numpy FP64) of consecutive particles of the 65,536-particle batch, "
                      "median of %d runs of ~%.0f s on a pool of %d processes; one thread: %.0f evals/s"
                      % (repeats, budget_s, workers, float(np.median(one))),
               one_thread_evals_per_s=float(np.median(one)), all_cores_evals_per_s=float(np.median(many)),
               runs_one_thread=one, runs_all_cores=many, cpu_model=model, nproc=avail)
    out["rjsmc"] = cpu_rjsmc_steps()
    return out


def cpu_rjsmc_steps(n_steps=2, n_per_sound=256):
    """The oracle's Algorithm 1 on one 256-particle sounding (R = 5, alpha = 0.5) for
    n_steps steps on one thread; the soundings/s figure assumes the step count of the
    GPU run of the same sounding (filled in by the caller)."""
    from oracle import algorithm1 as A1
    import warnings
    from oracle import em
    system = W.system()
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        K = em.make_K(system)
    y = em.forward(W.truth_three_layer(), system, K)[0]
    d = y + np.sqrt(em.noise_variance(y, system["eps_an"], system["eps_mn"])) * W.data_noise(1)
    t0 = time.perf_counter()
    A1.run(system, K, d[None, :], 1, n_per_sound, W.PRIOR, 0, max_steps=n_steps)
    dt = time.perf_counter() - t0
    return {"particles_per_sounding": n_per_sound, "steps_timed": n_steps, "seconds": dt,
            "seconds_per_step": dt / n_steps, "cores": 1}


def rjsmc_rate(torch, d, n_sound, n_per_sound, seed=0, move_prob=None, graph=False, kmax=None, noise=False,
               tune=False, **run_kw):
    """Soundings per second of complete Algorithm-1 runs (gamma 0 -> 1): n_sound soundings
    of n_per_sound particles each, alpha = 0.5, 5 moves per step, run together in the
    same launches (graph=True: one captured HIP graph per step, captured by a warm-up run
    and replayed by the timed run on the same driver, as when soundings are processed
    one run after another).  The soundings are copies of the synthetic sounding, or
    (noise=True) independent noise realisations of its response.  Wall clock includes the
    prior draw, every step and the per-step host check.  The spread over the replicate
    soundings of log Z of the best model and of the posterior probability of a chargeable
    model measures Monte Carlo accuracy."""
    from paper_2109_00661_amd import binding as B
    from paper_2109_00661_amd.rjsmc import RJSMCRun, UNIFORM_MOVES
    mp = UNIFORM_MOVES if move_prob is None else move_prob
    kc, km = kmax if kmax is not None else (W.PRIOR["kmax_cond"], W.PRIOR["kmax_charg"])
    system = W.system(kmax_cond=kc, kmax_charg=km)
    ctx = B.Context(system, precision="f64", max_particles=n_sound * n_per_sound)
    d0 = d.cpu().numpy()
    if noise:
        y_true = synth_response()
        s = np.sqrt(system["eps_an"] ** 2 + (system["eps_mn"] * y_true) ** 2)
        y = np.stack([y_true + s * W.data_noise(1000 + i) for i in range(n_sound)])
    else:
        y = np.tile(d0, (n_sound, 1))
    tuned = None
    if tune:
        warm = RJSMCRun(ctx, n_sound, n_per_sound, y, seed=seed + 99, move_prob=mp)
        warm.initialise()
        tuned, _ = ctx.autotune(warm.state, warm.y_obs, reps=3)
    if graph:
        # soundings processed one run after another on one driver: the warm-up run captures
        # the step graphs, the timed run replays them on a fresh prior population
        run = RJSMCRun(ctx, n_sound, n_per_sound, y, seed=seed + 99, move_prob=mp, graph=graph, **run_kw).run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run.rerun(seed)
    else:
        RJSMCRun(ctx, n_sound, n_per_sound, y, seed=seed + 99, move_prob=mp, graph=graph, **run_kw).run()   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run = RJSMCRun(ctx, n_sound, n_per_sound, y, seed=seed, move_prob=mp, graph=graph, **run_kw).run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = run.stats.cpu().numpy()
    probs = run.model_probabilities()
    p_ip = probs[:, (np.arange(probs.shape[1]) % (km + 1)) >= 1].sum(axis=1)
    lz = run.log_z.cpu().numpy()
    best = int(np.argmax(probs.mean(axis=0)))
    out = {"soundings_per_s": n_sound / dt, "n_sound": n_sound, "particles_per_sounding": n_per_sound,
           "steps": run.step, "seconds": dt, "graph": graph,
           "proposals_per_sounding": float(st[0].sum() / n_sound),
           "acceptance": float(st[1].sum() / max(st[0].sum(), 1)),
           "p_chargeable_mean": float(p_ip.mean()), "p_chargeable_sd": float(p_ip.std()),
           "best_model": best,
           "ll_max_median": float(np.median(run.ll.cpu().numpy().reshape(n_sound, n_per_sound).max(axis=1)))}
    if run_kw:
        out["sweeps_per_step_mean"] = float(np.mean(run.moves_per_step))
    if tuned is not None:
        out["tuning"] = tuned
    if n_sound > 1:
        fin = np.isfinite(lz[:, best])
        out["log_z_best_sd"] = float(np.std(lz[fin, best])) if fin.any() else None
        out["log_z_best_finite"] = int(fin.sum())
        # marginal evidence log p(y) = log (1/M) sum_k Z_k (uniform model prior), per replicate
        mx = np.max(np.where(np.isfinite(lz), lz, -np.inf), axis=1)
        lpy = mx + np.log(np.sum(np.exp(np.where(np.isfinite(lz), lz - mx[:, None], -np.inf)), axis=1)) - np.log(
            lz.shape[1])
        out["log_evidence_mean"] = float(np.mean(lpy))
        out["log_evidence_sd"] = float(np.std(lpy))
        # the same marginal evidence from the replicate's most populated model k*:
        # p(y) = p(k*) Z_k* / pi(k* | y), with pi(k* | y) = N_k* / N (Section 3.2.1)
        ks = np.argmax(probs, axis=1)
        lz_ks = lz[np.arange(n_sound), ks]
        lpy_pop = lz_ks - np.log(lz.shape[1]) - np.log(probs[np.arange(n_sound), ks])
        fin2 = np.isfinite(lpy_pop)
        out["log_evidence_pop_mean"] = float(np.mean(lpy_pop[fin2])) if fin2.any() else None
        out["log_evidence_pop_sd"] = float(np.std(lpy_pop[fin2])) if fin2.any() else None
        out["p_best_model_mean"] = float(np.mean(probs[:, best]))
        out["p_best_model_sd"] = float(np.std(probs[:, best]))
    return out


def rjsmc_legs():
    """The RJSMC measurements of the default run, by name."""
    from paper_2109_00661_amd.rjsmc import LANGEVIN_MOVES
    return {
        "single_sounding_256": lambda torch, d: rjsmc_rate(torch, d, 1, 256),
        "single_sounding_256_tuned_graph": lambda torch, d: rjsmc_rate(torch, d, 1, 256, graph=True, tune=True),
        "batched_64x256_rw": lambda torch, d: rjsmc_rate(torch, d, 64, 256, graph=True, tune=True),
        "batched_64x256_langevin": lambda torch, d: rjsmc_rate(torch, d, 64, 256, move_prob=LANGEVIN_MOVES,
                                                               graph=True, tune=True),
        "batched_64x256_adaptive_sweeps_tuned_scale": lambda torch, d: rjsmc_rate(
            torch, d, 64, 256, graph=True, tune=True, adapt_c=0.05, r_max=40, tune_scale=True),
        "uneven_512x1024_rw": lambda torch, d: rjsmc_rate(torch, d, 512, 1024, graph=True, kmax=(7, 4), noise=True,
                                                          tune=True),
    }


def accuracy_comparison(torch, d, sizes=(1024, 4096), reps=16, adapt_c=0.01, r_max=40, extras=False):
    """Random-walk against gradient-informed (Langevin) within-model moves on the same
    GPU, as a cost-versus-accuracy curve: `reps` replicate runs of the synthetic sounding
    (batched) for each particle count, with the adaptive number of sweeps (c = 0.01:
    every particle moves with probability 0.99, at most 40 sweeps), each within-model step
    bisected on trial proposals (random-walk scale toward acceptance 0.44, Langevin step
    toward 0.574), tuned tiles and step graphs.  Accuracy is the spread over replicates of
    the marginal log-evidence (from the most populated model's evidence and its posterior
    probability, and from the sum over models), of the best model's log-evidence and of
    its posterior probability; cost is soundings/s.  `at_equal_accuracy` gives, for the
    spread both samplers reach, each one's cheapest configuration that reaches it.
    extras: also the random walk at 512 particles with the adaptive birth and with
    particle recycling (8 populations, eager)."""
    from paper_2109_00661_amd.rjsmc import UNIFORM_MOVES, LANGEVIN_MOVES
    rows = []
    cases = [(name, mp, n, True, {}) for n in sizes
             for name, mp in (("random_walk", UNIFORM_MOVES), ("langevin", LANGEVIN_MOVES))]
    if extras:
        cases += [("random_walk_adaptive_birth", UNIFORM_MOVES, 512, True, {"zca_birth": True}),
                  ("random_walk_recycling_8", UNIFORM_MOVES, 512, False, {"recycle": 8})]
    for name, mp, n, graph, extra in cases:
        r = rjsmc_rate(torch, d, reps, n, move_prob=mp, graph=graph, tune=True, adapt_c=adapt_c, r_max=r_max,
                       tune_scale=True, **extra)
        row = {"moves": name, "particles_per_sounding": n, "replicates": reps, "graph": graph}
        row.update({k: r.get(k) for k in ("soundings_per_s", "steps", "sweeps_per_step_mean", "acceptance",
                                          "log_evidence_pop_mean", "log_evidence_pop_sd", "log_evidence_mean",
                                          "log_evidence_sd", "log_z_best_sd", "best_model", "p_best_model_mean",
                                          "p_best_model_sd", "p_chargeable_mean", "p_chargeable_sd",
                                          "ll_max_median")})
        print(json.dumps(row), file=sys.stderr, flush=True)
        rows.append(row)
    equal = {}
    for measure in ("log_evidence_pop_sd", "p_best_model_sd"):
        best = {}
        for m in ("random_walk", "langevin"):
            vals = [r[measure] for r in rows if r["moves"] == m and r[measure] is not None]
            best[m] = min(vals) if vals else None
        if None in best.values():
            continue
        target = max(best.values())                     # a spread both samplers reach
        pick = {}
        for m in ("random_walk", "langevin"):
            ok = [r for r in rows if r["moves"] == m and r[measure] is not None and r[measure] <= target]
            r = max(ok, key=lambda r: r["soundings_per_s"])
            pick[m] = {"particles_per_sounding": r["particles_per_sounding"], "soundings_per_s": r["soundings_per_s"],
                       measure: r[measure]}
        equal[measure] = {"common_spread": target, **pick,
                          "random_walk_over_langevin": pick["random_walk"]["soundings_per_s"]
                          / pick["langevin"]["soundings_per_s"]}
    return {"rows": rows, "at_equal_accuracy": equal}


def survey_run(torch, precision, move_prob, n_per_sound=2048, seed=0):
    """Complete RJSMC runs over the synthetic survey (2,000 soundings on 10 lines): wall
    clock, and how well the per-sounding log BFIPD separates the stations above the
    chargeable body (should be > 0) from the others (< 0)."""
    from paper_2109_00661_amd import binding as B
    from paper_2109_00661_amd.rjsmc import RJSMCRun
    truth, body, _, _ = W.survey()
    S = len(body)
    system = W.system()
    ref = B.Context(system, precision="f64")
    y_true = ref.forward(B.particles_to_device(truth)).cpu().numpy()
    ref.check()
    sd = np.sqrt(system["eps_an"][None, :] ** 2 + (system["eps_mn"] * y_true) ** 2)
    noise = np.stack([np.random.default_rng(5000 + i).standard_normal(y_true.shape[1]) for i in range(S)])
    y = y_true + sd * noise
    ctx = B.Context(system, precision=precision, max_particles=S * n_per_sound)
    run = RJSMCRun(ctx, S, n_per_sound, y, seed=seed, move_prob=move_prob, graph=True)
    run.initialise()
    tuned, _ = ctx.autotune(run.state, run.y_obs, reps=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run.run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    summ = ctx.summarize(run.state, S)
    lb = summ["log_bfipd"].cpu().numpy()
    # posterior predictive check: the data standardised to each station's PPD
    zs = np.abs(run.posterior_predictive()["z"].cpu().numpy())
    lz = run.log_z.cpu().numpy()
    km = ctx.kmax_charg
    true_model = truth["kappa"] * (km + 1) + truth["lambda_"]
    lz_true = lz[np.arange(S), true_model]
    st = run.stats.cpu().numpy()
    return {"precision": precision, "soundings": S, "particles_per_sounding": n_per_sound,
            "soundings_per_s": S / dt, "seconds": dt, "steps": run.step, "tuning": tuned,
            "acceptance": float(st[1].sum() / max(st[0].sum(), 1)),
            "detect_true_positive": float(np.mean(lb[body] > 0)),
            "detect_true_negative": float(np.mean(lb[~body] < 0)),
            "log_bfipd_median_body": float(np.median(lb[body])),
            "log_bfipd_median_outside": float(np.median(lb[~body])),
            "log_z_true_model_finite": int(np.isfinite(lz_true).sum()),
            "ppd_abs_z_median": float(np.median(zs)), "ppd_frac_within_1sd": float(np.mean(zs <= 1.0)),
            "ppd_frac_within_3sd": float(np.mean(zs <= 3.0)),
            "_log_bfipd": lb, "_log_z_true": lz_true}


def survey(torch, langevin=False):
    from paper_2109_00661_amd.rjsmc import UNIFORM_MOVES, LANGEVIN_MOVES
    runs = {"fp64_rw": survey_run(torch, "f64", UNIFORM_MOVES),
            "fp32_forward_rw": survey_run(torch, "f32", UNIFORM_MOVES)}
    if langevin:
        runs["fp64_langevin"] = survey_run(torch, "f64", LANGEVIN_MOVES)
    a, b = runs["fp64_rw"]["_log_bfipd"], runs["fp32_forward_rw"]["_log_bfipd"]
    fin = np.isfinite(a) & np.isfinite(b)
    za, zb = runs["fp64_rw"]["_log_z_true"], runs["fp32_forward_rw"]["_log_z_true"]
    zf = np.isfinite(za) & np.isfinite(zb)
    out = {k: {kk: vv for kk, vv in v.items() if not kk.startswith("_")} for k, v in runs.items()}
    out["fp32_vs_fp64"] = {"bfipd_sign_agreement": float(np.mean(np.sign(a) == np.sign(b))),
                           "log_bfipd_median_abs_diff": float(np.median(np.abs(a[fin] - b[fin]))) if fin.any() else None,
                           "log_z_true_median_abs_diff": float(np.median(np.abs(za[zf] - zb[zf]))) if zf.any() else None}
    return out


def reweight_rate(torch, d, steps, warmup, n_sound=2000, n_per_sound=2048):
    """Re-weight + within-model resampling (with the resampled copy) of survey-sized
    populations: n_sound soundings of n_per_sound prior particles with their
    log-likelihoods, each call from gamma = 0 (the two small fills that reset gamma and
    log Z are inside the timed region).  Algorithmic HBM bytes per particle: the counts,
    ll and every parameter row read once, the resampled rows, counts, ll and ancestor
    written once."""
    from paper_2109_00661_amd import binding as B
    system = W.system()
    n = n_sound * n_per_sound
    ctx = B.Context(system, precision="f64", max_particles=n)
    kc, km = ctx.kmax_cond, ctx.kmax_charg
    M = (kc + 1) * (km + 1)
    p = B.empty_device_population(n, kc, km, n_per_sound)
    ctx.init_prior(p, W.PRIOR, 11)
    y = d.reshape(1, -1).repeat(n_sound, 1).contiguous()
    ll = ctx.loglik(p, y)
    out = B.empty_device_population(n, kc, km, n_per_sound)
    ll_out = torch.empty_like(ll)
    gamma = torch.zeros(n_sound, dtype=torch.float64, device="cuda")
    log_z = torch.zeros((n_sound, M), dtype=torch.float64, device="cuda")
    anc = torch.empty(n, dtype=torch.int32, device="cuda")

    def call():
        gamma.zero_()
        log_z.zero_()
        ctx.reweight_resample(p, ll, out, ll_out, gamma, log_z, None, anc, 0.5, 3, 1, n_sound)

    ms, _ = time_calls(call, steps, warmup, torch)
    ctx.check()
    rows = 3 + 2 * kc + 2 * km                     # phi_b, log10 tau, c, phi, z, m, zm
    per_particle = (8 + 8 + 8 * rows) + (8 * rows + 8 + 8 + 4)
    return {"soundings": n_sound, "particles_per_sounding": n_per_sound, "ms_per_call": ms,
            "algorithmic_bytes_per_particle": per_particle,
            "hbm_gb_per_s": per_particle * n / (ms * 1e-3) / 1e9,
            "hbm_frac_of_8tb_s": per_particle * n / (ms * 1e-3) / 8e12,
            "gamma_mean": float(gamma.mean().item())}


def adjoint_rate(torch, d, steps, warmup):
    """Log-likelihood + gradient evaluations per second for 65,536 decoupled particles
    with 1-8 segments per partition (merged layers up to 15).  The context holds a
    workspace for the batch, so particles are split by their merged-layer count among the
    8-, 12- and 16-layer instantiations."""
    from paper_2109_00661_amd import binding as B
    system = W.system(kmax_cond=7, kmax_charg=7)
    ctx = B.Context(system, precision="f64", max_particles=N_PARTICLES)
    n = N_PARTICLES
    rng = np.random.default_rng(3)
    p = W.empty_particles(n, 7, 7)
    p["kappa"][:] = rng.integers(0, 8, n)
    p["lambda_"][:] = rng.integers(0, 8, n)
    P = W.PRIOR
    p["phi_b"][:] = rng.uniform(P["phi_lo"], P["phi_hi"], n)
    p["log10_tau"][:] = rng.uniform(P["ltau_lo"], P["ltau_hi"], n)
    p["c"][:] = rng.uniform(P["c_lo"], P["c_hi"], n)
    zc = np.sort(rng.uniform(0, P["z_max"], (7, n)), axis=0)
    zm = np.sort(rng.uniform(0, P["z_max"], (7, n)), axis=0)
    for r in range(7):
        p["z_cond"][r] = np.where(r < p["kappa"], zc[r], 0.0)
        p["z_charg"][r] = np.where(r < p["lambda_"], zm[r], 0.0)
    p["phi"][:] = rng.uniform(P["phi_lo"], P["phi_hi"], (7, n))
    p["m"][:] = rng.uniform(P["m_lo"], P["m_hi"], (7, n))
    dp = B.particles_to_device(p)
    ms, _ = time_calls(lambda: ctx.loglik_grad(dp, d), steps, warmup, torch)
    ms_f, _ = time_calls(lambda: ctx.loglik(dp, d), steps, warmup, torch)
    ctx.check()
    # the default prior (at most 4 conductivity and 3 chargeability interfaces, so at most
    # 8 merged layers): the register-resident instantiation of the reverse sweep
    ctx8 = B.Context(W.system(), precision="f64", max_particles=n)
    p8 = B.empty_device_population(n, ctx8.kmax_cond, ctx8.kmax_charg)
    ctx8.init_prior(p8, W.PRIOR, 5)
    ms8, _ = time_calls(lambda: ctx8.loglik_grad(p8, d), steps, warmup, torch)
    ctx8.check()
    return {"grad_evals_per_s": n / (ms * 1e-3), "ms_per_launch": ms, "forward_ms_same_population": ms_f,
            "grad_over_forward": ms / ms_f, "mean_merged_layers": float((p["kappa"] + p["lambda_"] + 1).mean()),
            "prior_population_ms_per_launch": ms8}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--extra", action="store_true", help="(the extra legs now run by default)")
    ap.add_argument("--quick", action="store_true",
                    help="skip the synthetic survey and the random-walk / Langevin comparison")
    ap.add_argument("--survey", action="store_true",
                    help="the synthetic survey also with Langevin moves (FP64 and FP32-forward random walk run "
                         "by default)")
    ap.add_argument("--compare", action="store_true",
                    help="the random-walk / Langevin comparison at 512 to 9,600 particles per sounding and with "
                         "the adaptive birth and recycling (1,024 and 4,096 run by default; minutes)")
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the 65,536-particle forward+loglik launches (for profiling)")
    ap.add_argument("--reweight-only", action="store_true",
                    help="time only re-weight/re-sample on 2,000 x 2,048 particles (for profiling)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="time only the 65,536-particle log-likelihood gradient launches (for profiling)")
    ap.add_argument("--rjsmc-leg", default=None,
                    help="run only this RJSMC leg (e.g. single_sounding_256_tuned_graph) and print it (profiling)")
    ap.add_argument("--precision", choices=("f64", "f32"), default="f64",
                    help="precision of the headline forward (f32: the FP32 variant, for its profile)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB before timing, as the "
                         "reference for hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path runs on a single MI355X; "
              "multi-GPU sharding by sounding is a design note only.", file=sys.stderr)
        sys.exit(2)

    # the CPU baseline first: its process pool forks, which must happen before the GPU is used
    profiling_leg = args.reweight_only or args.adjoint_only or args.rjsmc_leg or args.headline_only
    cpu = None if (args.no_cpu or profiling_leg) else cpu_baseline()

    import torch
    from paper_2109_00661_amd import binding as B

    if args.reweight_only:
        copy_calibration(torch, args.copy_calibration_mib)
        print(json.dumps({"reweight_resample": reweight_rate(torch, synth_data(torch), args.steps, args.warmup)}),
              flush=True)
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_rate(torch, synth_data(torch), args.steps, args.warmup)}), flush=True)
        return
    if args.rjsmc_leg:
        legs = rjsmc_legs()
        if args.rjsmc_leg not in legs:
            print("unknown leg; choose from " + ", ".join(legs), file=sys.stderr)
            sys.exit(2)
        print(json.dumps({args.rjsmc_leg: legs[args.rjsmc_leg](torch, synth_data(torch))}), flush=True)
        return
    system = W.system(kmax_cond=N_LAYERS - 1, kmax_charg=0)
    ctx = B.Context(system, precision=args.precision)
    d = synth_data(torch)
    p = B.particles_to_device(W.merged_population(N_PARTICLES, N_LAYERS, seed=2, kc=N_LAYERS - 1))
    ll = torch.empty(N_PARTICLES, dtype=torch.float64, device="cuda")

    copy_calibration(torch, args.copy_calibration_mib)
    ms, wall = time_calls(lambda: ctx.loglik(p, d, out=ll), args.steps, args.warmup, torch)
    ctx.check()
    evals = N_PARTICLES / (ms * 1e-3)
    flop = nominal_flop_per_eval(N_LAYERS) * N_PARTICLES
    achieved = flop / (ms * 1e-3) / 1e12
    f32 = args.precision == "f32"
    peak = FP32_VECTOR_PEAK_TFLOPS if f32 else FP64_VECTOR_PEAK_TFLOPS
    out = {
        "metric": "forward+loglik evals/sec (65k particles, Cole-Cole); RJSMC soundings/sec",
        "value": evals, "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": "forward+loglik, 65,536 five-layer Cole-Cole particles from the prior, "
                               "40 frequencies x 120-point J1 filter x 20 gates, " + ("FP32" if f32 else "FP64"),
                   "particles": N_PARTICLES, "layers": N_LAYERS},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None if f32 else measured_traffic(),
                     "traffic_unit": "HBM bytes per launch",
                     "kernel": "forward_kernel<%s,4,1>" % ("float" if f32 else "double"), "flop_per_launch": flop},
        "wall_s_timed": wall,
    }
    if args.headline_only:
        print(json.dumps(out), flush=True)
        return
    progress = lambda what: print("[bench] %s" % what, file=sys.stderr, flush=True)
    ctx32 = B.Context(system, precision="f32")
    ms32, _ = time_calls(lambda: ctx32.loglik(p, d, out=ll), args.steps, args.warmup, torch)
    a32 = flop / (ms32 * 1e-3) / 1e12
    out["fp32"] = {"evals_per_s": N_PARTICLES / (ms32 * 1e-3), "ms_per_step": ms32,
                   "nominal_tflops": a32, "frac_of_fp32_peak": a32 / FP32_VECTOR_PEAK_TFLOPS}
    progress("adjoint")
    out["adjoint"] = adjoint_rate(torch, d, max(3, args.steps // 4), 1)
    progress("reweight/resample 2,000 x 2,048")
    out["reweight_resample_2000x2048"] = reweight_rate(torch, d, max(3, args.steps // 4), 1)
    out["rjsmc"] = {}
    for name, leg in rjsmc_legs().items():
        progress("rjsmc " + name)
        out["rjsmc"][name] = leg(torch, d)
    if not args.quick:
        progress("survey 2,000 x 2,048")
        out["survey"] = survey(torch, langevin=args.survey)
        progress("random walk vs Langevin")
        out["moves_accuracy_comparison"] = (accuracy_comparison(torch, d, sizes=(512, 1024, 2048, 4096, 9600),
                                                                extras=True)
                                            if args.compare else accuracy_comparison(torch, d))
    if cpu is not None:
        # the oracle's RJSMC rate: its seconds per step times the GPU run's step count
        ref = out["rjsmc"].get("single_sounding_256")
        if ref:
            cpu["rjsmc"]["steps_assumed"] = ref["steps"]
            cpu["rjsmc"]["soundings_per_s"] = 1.0 / (cpu["rjsmc"]["seconds_per_step"] * ref["steps"])
            cpu["rjsmc"]["extrapolation"] = ("seconds per Algorithm-1 step of the first %d steps x the %d steps of "
                                             "the GPU run of the same sounding" % (cpu["rjsmc"]["steps_timed"],
                                                                                    ref["steps"]))
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
