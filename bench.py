"""Benchmark: MFM hydro steps of the 2.1M-particle Sedov blast on one MI355X.

Workload: 128^3 particles, lattice + 0.1-spacing jitter, rho = 1, P = 1e-6, unit
energy deposited kernel-weighted in the central 33 particles, gamma = 5/3,
N_NGB = 32, MFM scheme.  Each timed step is one mfm_step: cell build (sort),
density / smoothing-length loop, neighbour lists, gradients + time step,
fluxes, update -- the whole hot path, inputs resident in HBM.

Metric: pair interactions per second over the gradient and flux loops,
(gradient pairs + flux faces) / (t_gradients + t_fluxes), with the loop times
from HIP events the library records on its own stream; ms per full step is
reported beside it.

The JSON line also carries
  roofline     -- the dominant kernel (the flux loop) against the FP64 vector
                  peak: algorithmic flops per launch / mean launch time;
  cpu_baseline -- the FP64 CPU oracle timed on the host on one full step of
                  the same particle set (density, gradients, fluxes), all
                  host threads.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP64 operations per face of the flux loop (add, sub, mul, div,
# sqrt and pow count 1, a fused multiply-add 2; comparisons and selects 0).
# The count runs over the stages of one face: separation and kernel weights,
# A_ij, half-step prediction and extrapolation, pairwise limiter, face-frame
# states, Riemann set-up, sampling (MFV) and flux assembly, accumulation; each
# Newton iteration of the Riemann solve adds FLOPS_NEWTON_ITER.
FLOPS_FACE = {"mfm": 388, "mfv": 458}
FLOPS_NEWTON_ITER = 30
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=128, help="particles per axis")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--scheme", default="mfm", choices=["mfm", "mfv"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    return ap.parse_args()


def log(msg, args):
    if not args.quiet:
        print(msg, file=sys.stderr, flush=True)


def cpu_baseline(st, scheme):
    """The oracle (unchanged) on one step of the same set; pair interactions/s."""
    import numpy as np

    import oracle

    cfg = {"scheme": scheme}
    t0 = time.perf_counter()
    d, _ = oracle.density(cfg, st["x"], st["y"], st["z"], st["H"])
    t1 = time.perf_counter()
    g, c2 = oracle.gradients(cfg, st["x"], st["y"], st["z"], d["H"], d["V"], st["m"], st["vx"],
                             st["vy"], st["vz"], st["U"])
    t2 = time.perf_counter()
    dt = float(np.min(g["dt_i"]))
    f, c3 = oracle.fluxes(cfg, st["x"], st["y"], st["z"], d["H"], d["V"], g["rho"], st["vx"],
                          st["vy"], st["vz"], g["P"], g["B"], g["grad"], dt)
    t3 = time.perf_counter()
    pairs = c2["grad_pairs"] + c3["faces"]
    threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    return {
        "value": pairs / ((t2 - t1) + (t3 - t2)),
        "unit": "pair interactions/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"one step (density, gradients, fluxes) of the full {len(st['x'])}-particle "
                   f"set; density {t1 - t0:.2f} s, gradients {t2 - t1:.2f} s, "
                   f"fluxes {t3 - t2:.2f} s"),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the library "
              "runs on a single GPU and has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2211_12243_amd import mfm
    from paper_2211_12243_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    t = time.perf_counter()
    st = W.sedov(n=args.n, seed=3)
    N = len(st["x"])
    log(f"[bench] sedov n={args.n}^3 ({N} particles) made in {time.perf_counter() - t:.1f}s", args)
    params = mfm.params_from_dict({"scheme": args.scheme}, precision=args.precision)
    ctx = mfm.Context(params, N)
    ps = mfm.ParticleSet(st, ids=False)
    for w in range(args.warmup):
        dt = mfm.mfm_step(ctx, ps, 1.0)
        log(f"[bench] warmup step {w} dt={dt:.3e}", args)
    mfm.mfm_reset_counters(ctx)
    mfm.mfm_enable_timing(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        dt = mfm.mfm_step(ctx, ps, 1.0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    times = mfm.mfm_kernel_times(ctx)
    diag = mfm.mfm_diagnostics(ctx, ps)
    K = args.steps
    log(f"[bench] {K} steps in {t1 - t0:.3f}s; stages {times}", args)
    log(f"[bench] diag {diag}", args)
    t_grad = times["gradients"][0] / 1e3
    t_flux = times["fluxes"][0] / 1e3
    pairs = diag["grad_pairs"] + diag["faces"]
    value = pairs / (t_grad + t_flux)
    ms_step = (t1 - t0) / K * 1e3
    # dominant kernel: the flux loop
    n_launch = max(times["fluxes"][1], 1)
    mean_s = t_flux / n_launch
    flops_launch = (diag["faces"] * FLOPS_FACE[args.scheme]
                    + diag["riemann_iters"] * FLOPS_NEWTON_ITER) / n_launch
    peak = PEAK_FP64_TFLOPS if args.precision == "fp64" else PEAK_FP32_TFLOPS
    achieved = flops_launch / mean_s / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None,
                "kernel": "fluxes_k", "mean_launch_ms": mean_s * 1e3,
                "flops_per_launch": flops_launch}
    out = {
        "metric": "pair interactions/s (grad+flux) & hydro-step ms, 2.1M Sedov, mixed vs FP64",
        "value": value,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"sedov {args.n}^3 MFM blast (lattice + 0.1 jitter, P=1e-6, "
                               f"E=1 in central 33)", "particles": N, "scheme": args.scheme,
                   "precision": args.precision, "n_ngb": 32, "gamma": 5.0 / 3.0},
        "stage_ms_per_step": {k: v[0] / K for k, v in times.items()},
        "pairs_per_step": {"gradient": diag["grad_pairs"] / K, "flux_faces": diag["faces"] / K,
                           "newton_iters_per_face": diag["riemann_iters"] / max(diag["faces"], 1)},
        "roofline": roofline,
    }
    ctx.close()
    del ps
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on one step of the same set", args)
        out["cpu_baseline"] = cpu_baseline(st, args.scheme)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
