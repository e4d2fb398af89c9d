"""Benchmark of the RJSMC hot path on one MI355X.

Headline: forward model + log-likelihood evaluations per second for 65,536 particles,
each a five-layer Cole-Cole model drawn from the prior ranges, with the 40-frequency /
120-point J1 / 20-gate central-loop system (FP64).  One step = one rjsmc_loglik launch
over the whole batch; inputs are resident in HBM before the timed region.

Prints one JSON line.  Options: --steps K --warmup W --gpus N (only 1 is supported)
--no-cpu (skip the CPU oracle baseline) --extra (also time FP32 and the other calls).
"""
import argparse
import json
import os
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


def nominal_flop_per_eval(n_layers, n_freq=40, n_hankel=120):
    return n_freq * n_hankel * n_layers * FLOP_PER_LAYER_STEP


def synth_data(torch):
    """Synthetic sounding: the three-layer truth through the forward model plus noise
    with the standard deviation of the noise model at the response."""
    from paper_2109_00661_amd import binding as B
    system = W.system(kmax_cond=2, kmax_charg=0)
    ctx = B.Context(system, precision="f64")
    y = ctx.forward(B.particles_to_device(W.truth_three_layer_merged())).cpu().numpy()[0]
    ctx.check()
    s = np.sqrt(system["eps_an"] ** 2 + (system["eps_mn"] * y) ** 2)
    return torch.as_tensor(y + s * W.data_noise(1), device="cuda")


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


def cpu_baseline(system, d_np, budget_s=15.0):
    """The oracle as it stands, on a bounded sample of the same workload."""
    import warnings
    from oracle import em
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        K = em.make_K(system)
    p = W.merged_population(N_PARTICLES, N_LAYERS, seed=2, kc=N_LAYERS - 1)
    n_done = 0
    t0 = time.perf_counter()
    chunk = 64
    while time.perf_counter() - t0 < budget_s and n_done < N_PARTICLES:
        em.loglik(p, system, K, d_np, range(n_done, min(n_done + chunk, N_PARTICLES)))
        n_done = min(n_done + chunk, N_PARTICLES)
    dt = time.perf_counter() - t0
    return dict(value=n_done / dt, unit="evals/s", cores=1, kind="oracle",
                sample="first %d of the 65,536 particles (numpy FP64, one thread), %.1f s" % (n_done, dt))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--extra", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path runs on a single MI355X; "
              "multi-GPU sharding by sounding is a design note only.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2109_00661_amd import binding as B

    system = W.system(kmax_cond=N_LAYERS - 1, kmax_charg=0)
    ctx = B.Context(system, precision="f64")
    d = synth_data(torch)
    p = B.particles_to_device(W.merged_population(N_PARTICLES, N_LAYERS, seed=2, kc=N_LAYERS - 1))
    ll = torch.empty(N_PARTICLES, dtype=torch.float64, device="cuda")

    ms, wall = time_calls(lambda: ctx.loglik(p, d, out=ll), args.steps, args.warmup, torch)
    ctx.check()
    evals = N_PARTICLES / (ms * 1e-3)
    flop = nominal_flop_per_eval(N_LAYERS) * N_PARTICLES
    achieved = flop / (ms * 1e-3) / 1e12
    out = {
        "metric": "forward+loglik evals/sec (65k particles, Cole-Cole); RJSMC soundings/sec",
        "value": evals, "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "forward+loglik, 65,536 five-layer Cole-Cole particles from the prior, "
                               "40 frequencies x 120-point J1 filter x 20 gates, FP64",
                   "particles": N_PARTICLES, "layers": N_LAYERS},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "kernel": "forward_kernel<8,double>", "flop_per_launch": flop},
        "wall_s_timed": wall,
    }
    if args.extra:
        ctx32 = B.Context(system, precision="f32")
        ms32, _ = time_calls(lambda: ctx32.loglik(p, d, out=ll), args.steps, args.warmup, torch)
        out["fp32"] = {"evals_per_s": N_PARTICLES / (ms32 * 1e-3), "ms_per_step": ms32}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(system, d.cpu().numpy())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
