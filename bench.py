"""Benchmark: MFM hydro steps of the 2.1M-particle Sedov blast on one MI355X.

Workload: 128^3 particles, lattice + 0.1-spacing jitter, rho = 1, P = 1e-6, unit
energy deposited kernel-weighted in the central 33 particles, gamma = 5/3,
N_NGB = 32, MFM scheme.  Each timed step is one mfm_step: cell build (sort),
neighbour search, density / smoothing-length loop, gradients + time step,
fluxes, update -- the whole hot path, inputs resident in HBM.

Variants, each from the same initial set with the same warm-up:
  fp64           all pair arithmetic in FP64 (the paper's precision);
  mixed          FP32 pair arithmetic, FP64 accumulators and checks, faces
                 across strong jumps in FP64;
  mixed_learned  mixed, with the Riemann iteration started from the guess
                 network (trained first, on faces dumped from other sets).
The reported value is the headline variant's (default fp64); every variant's
rate, stage times and per-kernel roofline fractions are in "variants".

Metric: pair interactions per second over the gradient and flux loops,
(gradient pairs + flux faces) / (t_gradients + t_fluxes), with the loop times
from HIP events the library records on its own stream (the flux loop's time
covers both of its passes and the clear and fold of its partial sums); ms per
full step is reported beside it.

The JSON line also carries
  roofline     -- the dominant kernel (the flux loop's first pass, fluxes_k)
                  against the vector ALU peak: the oracle's operation count
                  per face times the faces it solves, over its mean launch time;
  cpu_baseline -- the FP64 CPU oracle timed on the host on one full step of
                  the same particle set (density, gradients, fluxes) with all
                  host threads, single-thread steps of two smaller sets, the
                  CPU model, and each field's error at step 1 against it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of the loops, from the oracle's operation counter
# (oracle/opcount.cpp: the oracle compiled with a number type that counts
# every add, multiply, divide, square root and power; python -m
# oracle.opcount 128 prints these; tests/test_opcount.py checks them):
# flops per face of the flux loop, mean over a 20000-face sample of the first
# step of the 128^3 Sedov set (Newton iterations included), and flops per
# ordered pair of the gradient loop (limiter and time step included).
FLOPS_PER_FACE = {"mfm": 450.29, "mfv": 537.29}
FLOPS_PER_GRAD_PAIR = 151.0
# Algorithmic HBM bytes per particle: the fields a loop must read and write
# once (FP64 path):
#   cells     key + order (8 B), gather and write-back of the 11-double state
#             (176 B), cell tables: 184 B
#   density   x, y, z, H read, H, V, rho, P, c, ncond written: 80 B
#   gradients the density loop's record (11 doubles) read, B (6), grad (15),
#             dt_i, ncond written: 288 B
#   fluxes    B, grad, primitives, position, V, 1/H read (32 doubles), dQ (5)
#             written: 296 B
#   search    position and H read (32 B), the candidate count and the list
#             written (index + r^2, 12 B per candidate; 35 per particle on the
#             128^3 Sedov set): 456 B
BYTES_PER_PARTICLE = {"cells": 184, "density": 80, "gradients": 288, "fluxes": 296,
                      "search": 456}
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_TBS = 8.0


VARIANTS = ("fp64", "mixed", "mixed_learned")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=128, help="particles per axis")
    ap.add_argument("--variants", default=",".join(VARIANTS),
                    help="comma-separated subset of " + ", ".join(VARIANTS))
    ap.add_argument("--headline", default="fp64", choices=VARIANTS,
                    help="variant whose rate is the reported value")
    ap.add_argument("--scheme", default="mfm", choices=["mfm", "mfv"])
    ap.add_argument("--train-steps", type=int, default=6000)
    ap.add_argument("--train-records", type=float, default=1e7,
                    help="size of the guess network's record set (gated faces all kept)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--clustered", type=int, default=256,
                    help="particles per axis of the clustered-gas leg (0: skip it)")
    ap.add_argument("--rung-base", type=int, default=32,
                    help="individual-step leg: base step in units of the global step (0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy a buffer of this many MiB on the device (a kernel of "
                         "known traffic, to calibrate hardware byte counters)")
    ap.add_argument("--no-small-configs", dest="small_configs", action="store_false",
                    help="skip the 16^3 shock tube and 64^3 shear-layer timings")
    ap.add_argument("--no-error-growth", dest="error_growth", action="store_false",
                    help="skip the multi-step comparison with the oracle (CPU leg)")
    ap.add_argument("--quiet", action="store_true")
    return ap.parse_args()


FLUX_SOURCES = ("paper_2211_12243_amd/csrc/fluxes.hip", "paper_2211_12243_amd/csrc/mfm_internal.h",
                "paper_2211_12243_amd/csrc/mlp_device.h", "include/mfm.h")


def flux_traffic(variant):
    """HBM bytes per launch of fluxes_k recorded in profiles/traffic_sedov128.md
    from rocprofv3 FETCH_SIZE and WRITE_SIZE, or None when that file is absent
    or was taken from different flux-kernel sources than the ones built now."""
    import hashlib
    import re

    path = os.path.join(ROOT, "profiles", "traffic_sedov128.md")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in FLUX_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    with open(path) as fh:
        for line in fh:
            m = re.match(r"traffic (\w+): (\d+) bytes per launch of fluxes_k; flux sources "
                         r"sha256 ([0-9a-f]+)", line.strip())
            if m and m.group(1) == variant and m.group(3) == h.hexdigest():
                return float(m.group(2))
    return None


def log(msg, args):
    if not args.quiet:
        print(msg, file=sys.stderr, flush=True)


SINGLE_THREAD_SNIPPET = """
import json, sys, time
sys.path.insert(0, %r)
import oracle
from paper_2211_12243_amd import workloads as W
out = {}
for name, st, cfg in (("sod16_mfv", W.sod(n=16, seed=1), {"scheme": "mfv"}),
                      ("kh64_mfv", W.kh(n=64, seed=2), {"scheme": "mfv"})):
    t0 = time.perf_counter()
    oracle.step(cfg, st, 1.0)
    out[name] = time.perf_counter() - t0
print(json.dumps(out))
"""


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def field_errors(gpu, d, g, f, mixed):
    """Step-1 error of each field against the oracle: max_i |gpu - ref| over
    max_i |ref| per field (gradients per field as vectors, B as a matrix);
    the flux sums per particle against the particle's own scales (mixed:
    momentum against |s_p|, energy against s_E + c |s_p|)."""
    import numpy as np

    def rel(a, b):
        den = np.abs(b).max()
        return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())

    ref = {"H": d["H"], "V": d["V"], "rho": g["rho"], "P": g["P"], "c": g["c"],
           "ncond": g["ncond"], "dt_i": g["dt_i"]}
    out = {k: rel(gpu[k], v) for k, v in ref.items()}
    out["B"] = rel(gpu["B"], g["B"])
    out["grad"] = max(rel(gpu["grad"][3 * q:3 * q + 3], g["grad"][3 * q:3 * q + 3])
                      for q in range(5))
    s = f["scale"]
    diff = np.abs(gpu["dQ"] - f["dQ"])
    den = s.copy()
    if mixed:
        sp = np.sqrt((s[1:4] ** 2).sum(0))
        den[1:4] = sp[None, :]
        den[4] = s[4] + g["c"] * sp
    names = ("dQ_mass", "dQ_px", "dQ_py", "dQ_pz", "dQ_E")
    for k in range(5):
        m = den[k] > 0
        out[names[k]] = float((diff[k][m] / den[k][m]).max()) if m.any() else 0.0
    return out


def cpu_baseline(st, scheme, step1_fields):
    """The oracle (unchanged) on one step of the same set; pair interactions/s.
    Also: the single-thread time of one oracle step of the 16^3 shock tube and
    the 64^3 shear layers (a child process with one OpenMP thread), the CPU
    model, and the GPU variants' step-1 errors against this step."""
    import subprocess

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
    env = dict(os.environ, OMP_NUM_THREADS="1")
    single = None
    try:
        r = subprocess.run([sys.executable, "-c", SINGLE_THREAD_SNIPPET % ROOT], env=env,
                           capture_output=True, text=True, timeout=120)
        if r.returncode == 0:
            single = {k + "_step_s": v for k, v in json.loads(r.stdout.strip().splitlines()[-1]).items()}
    except (subprocess.TimeoutExpired, ValueError, IndexError):
        single = None
    errors = {v: field_errors(fl, d, g, f, v != "fp64") for v, fl in step1_fields.items()}
    return {
        "value": pairs / ((t2 - t1) + (t3 - t2)),
        "unit": "pair interactions/s",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": (f"one step (density, gradients, fluxes) of the full {len(st['x'])}-particle "
                   f"set; density {t1 - t0:.2f} s, gradients {t2 - t1:.2f} s, "
                   f"fluxes {t3 - t2:.2f} s"),
        "single_thread": single,
        "step1_errors": errors,
    }


def step1_fields(args, st, variant):
    """The GPU's fields after density, gradients and fluxes of the first step
    (host copies, original particle order), for the comparison with the oracle."""
    import numpy as np
    import torch

    from paper_2211_12243_amd import mfm

    precision = "fp64" if variant == "fp64" else "mixed"
    ctx = mfm.Context(mfm.params_from_dict({"scheme": args.scheme}, precision=precision),
                      len(st["x"]))
    ps = mfm.ParticleSet(st)
    mfm.run_pipeline(ctx, ps, 1.0, update=False)
    torch.cuda.synchronize()
    ids = ps["id"].cpu().numpy()
    out = {}
    for k in ("H", "V", "rho", "P", "c", "ncond", "dt_i", "B", "grad", "dQ"):
        t = ps[k].cpu().numpy()
        a = np.empty_like(t)
        a[..., ids] = t
        out[k] = a
    ctx.close()
    del ps
    return out


def train_guess(args, c4, log_):
    """The guess network's training set and training.  Face records dumped by
    the plain solver from the shear layers (64^3, 10 steps per scheme), a
    Sedov blast of the benchmark's recipe with another seed (20 steps after
    two warm-up steps) and the clustered gas (one step): the faces that pass
    the guess gate (all of them, or a uniform sample of half the set's share
    where there are more) and a uniform sample of the others, about a third
    of --train-records per set.  Split 90/10 (seeded); the network trains on
    the gated records of the 90%.  Also: a network trained without the Sedov
    records, scored on them (leave one set out).  Returns (state, info)."""
    import torch

    from paper_2211_12243_amd import learned, mfm
    from paper_2211_12243_amd import workloads as W

    t0 = time.perf_counter()
    sets = [("kh64_mfv_fp64", lambda: W.kh(n=64, seed=2), "mfv", "fp64", 0, 10),
            ("kh64_mfm_mixed", lambda: W.kh(n=64, seed=2), "mfm", "mixed", 0, 10),
            (f"sedov{args.n}_mfm_mixed", lambda: W.sedov(n=args.n, seed=17), "mfm", "mixed",
             2, 20),
            ("clustered_mfm_mixed", lambda: c4, "mfm", "mixed", 0, 1)]
    per_set = args.train_records / 3.0
    rows, info_sets = {}, {}
    for k, (name, make, scheme, precision, skip, steps) in enumerate(sets):
        st = make()
        n = len(st["x"])
        share = per_set / (2 if name.startswith("kh64") else 1)
        rate = min(1.0, 0.5 * share / (14.5 * n * steps))
        ctx = mfm.Context(mfm.params_from_dict({"scheme": scheme}, precision=precision), n)
        ps = mfm.ParticleSet(st, ids=False)
        for _ in range(skip):
            mfm.mfm_step(ctx, ps, 1.0)
        col = learned.Collector(ctx, 24 * n, rate, seed=100 + k,
                                gated_budget=int(0.5 * share / steps))
        for _ in range(steps):
            col.step(ps)
        rows[name] = col.rows()
        info_sets[name] = {"particles": n, "steps": steps, "faces": col.faces,
                           "gated": col.gated, "kept": int(rows[name].shape[0]),
                           "truncated": col.truncated}
        log_(f"[bench] guess records from {name}: {info_sets[name]}")
        del col, ps
        ctx.close()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    parts = {name: learned.split(r, 0.9, seed=7) for name, r in rows.items()}
    train_rows = torch.cat([p[0] for p in parts.values()])
    test_rows = {name: p[1] for name, p in parts.items()}
    stt, losses = learned.train(train_rows, args.train_steps, batch=16384, lr=3e-3, seed=0)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    held_out = {name: learned.rms_error(stt, r) for name, r in test_rows.items()}
    sedov = sets[2][0]
    loo_train = torch.cat([p[0] for name, p in parts.items() if name != sedov])
    loo, _ = learned.train(loo_train, args.train_steps, batch=16384, lr=3e-3, seed=0)
    info = {"records": int(sum(r.shape[0] for r in rows.values())),
            "train_records": int(train_rows.shape[0]),
            "train_gated": int(learned.usable(train_rows).sum()),
            "sets": info_sets, "dump_s": t1 - t0, "train_s": t2 - t1,
            "steps": args.train_steps, "batch": 16384,
            "loss_first": losses[0], "loss_last": losses[-1],
            "held_out_rms_ln_pstar": held_out,
            "leave_out_sedov_rms_ln_pstar": learned.rms_error(loo, test_rows[sedov])}
    log_(f"[bench] trained guess network: {info}")
    del rows, parts, train_rows, test_rows, loo_train
    return stt, info


def run_variant(args, st, variant, mlp_state, log_):
    """Warm-up and timed steps of one variant on a fresh copy of the set."""
    import torch

    from paper_2211_12243_amd import mfm

    precision = "fp64" if variant == "fp64" else "mixed"
    guess = 1 if variant == "mixed_learned" else 0
    params = mfm.params_from_dict({"scheme": args.scheme, "guess": guess}, precision=precision)
    ctx = mfm.Context(params, len(st["x"]))
    if guess:
        mfm.mfm_mlp_attach(ctx, mlp_state)
    ps = mfm.ParticleSet(st, ids=False)
    for w in range(args.warmup):
        dt = mfm.mfm_step(ctx, ps, 1.0)
        log_(f"[bench] {variant} warmup step {w} dt={dt:.3e}")
    mfm.mfm_reset_counters(ctx)
    mfm.mfm_enable_timing(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mfm.mfm_step(ctx, ps, 1.0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    times = mfm.mfm_kernel_times(ctx)
    diag = mfm.mfm_diagnostics(ctx, ps)
    diag["n"] = ps.n
    newton = None
    if precision == "mixed":
        # one more step with every face dumped: Newton steps per face (mean,
        # 99th percentile), over all faces and over those the guess gate picks
        from paper_2211_12243_amd import learned

        mfm.mfm_reset_counters(ctx)
        col = learned.Collector(ctx, 24 * ps.n, None, seed=0)
        col.step(ps)
        newton = learned.iteration_stats(col.rows())
        d1 = mfm.mfm_diagnostics(ctx)
        newton["guess_fallbacks"] = d1["guess_fallback"]
        newton["guess_fallback_rate"] = (d1["guess_fallback"] / newton["gated"]
                                         if guess and newton["gated"] else 0.0)
        del col
    ctx.close()
    K = args.steps
    t_grad = times["gradients"][0] / 1e3
    t_flux = times["fluxes"][0] / 1e3  # the whole flux loop: both passes, clear and fold
    pairs = diag["grad_pairs"] + diag["faces"]
    peak = PEAK_FP64_TFLOPS if precision == "fp64" else PEAK_FP32_TFLOPS
    N = diag["n"]

    def mean_launch(stage):
        return times[stage][0] / 1e3 / max(times[stage][1], 1)

    # the dominant kernel: the flux loop's first pass (every face but those
    # handed to the FP64 second pass), op-counted flops per launch
    n_launch = max(times["flux_kernel"][1], 1)
    faces_main = (diag["faces"] - diag["hard_faces"]) / n_launch
    t_main = mean_launch("flux_kernel")
    flops_main = faces_main * FLOPS_PER_FACE[args.scheme]
    achieved = flops_main / t_main / 1e12
    kernels = {}
    for stage, unit_flops in (("gradients", FLOPS_PER_GRAD_PAIR * diag["grad_pairs"] / K),
                              ("fluxes", FLOPS_PER_FACE[args.scheme] * diag["faces"] / K),
                              ("density", None), ("cells", None), ("search", None)):
        t = times[stage][0] / 1e3 / K
        hbm = BYTES_PER_PARTICLE[stage] * N / t / 1e12
        e = {"ms": t * 1e3, "hbm_TBs": hbm, "hbm_frac": hbm / PEAK_HBM_TBS}
        if unit_flops is not None:
            e["TFLOPs"] = unit_flops / t / 1e12
            e["valu_frac"] = e["TFLOPs"] / peak
        e["frac"] = max(e.get("valu_frac", 0.0), e["hbm_frac"])
        kernels[stage] = e
    res = {
        "value": pairs / (t_grad + t_flux),
        "ms_per_step": (t1 - t0) / K * 1e3,
        "stage_ms_per_step": {k: v[0] / K for k, v in times.items()},
        "pairs_per_step": {"gradient": diag["grad_pairs"] / K, "flux_faces": diag["faces"] / K},
        "newton_iters_per_face": diag["riemann_iters"] / max(diag["faces"], 1),
        "fp64_pass_faces_frac": diag["hard_faces"] / max(diag["faces"], 1),
        "guess_fallback_frac": diag["guess_fallback"] / max(diag["faces"], 1),
        "newton_after": newton,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": flux_traffic(variant),
                     "kernel": "fluxes_k", "mean_launch_ms": t_main * 1e3,
                     "flops_per_launch": flops_main,
                     "flops_per_face": FLOPS_PER_FACE[args.scheme]},
        "kernels": kernels,
        "conserved_after": {k: diag[k] for k in ("mass", "px", "py", "pz", "energy")},
    }
    log_(f"[bench] {variant}: {res}")
    return res


def run_rungs(args, st, ms_global, log_):
    """The same set on individual time steps (FP64): after the warm-up, one
    base step of rung_base global steps' length (the global step of the last
    warm-up step), against the global steps that cover the same time."""
    import torch

    from paper_2211_12243_amd import mfm

    params = mfm.params_from_dict({"scheme": args.scheme}, precision="fp64")
    ctx = mfm.Context(params, len(st["x"]))
    ps = mfm.ParticleSet(st, ids=False)
    dt = 0.0
    for _ in range(args.warmup):
        dt = mfm.mfm_step(ctx, ps, 1.0)
    dt0 = args.rung_base * dt
    mfm.mfm_reset_counters(ctx)
    mfm.mfm_enable_timing(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nsub, r = mfm.mfm_step_rungs(ctx, ps, dt0)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    times = mfm.mfm_kernel_times(ctx)
    diag = mfm.mfm_diagnostics(ctx, ps)
    counts = torch.bincount(r.long()).cpu().tolist()
    ctx.close()
    res = {
        "variant": "fp64",
        "base_step": dt0,
        "base_step_in_global_steps": args.rung_base,
        "sub_steps": nsub,
        "ms_per_base_step": ms,
        "global_ms_same_time": ms_global * args.rung_base,
        "speedup": ms_global * args.rung_base / ms,
        "particles_per_rung": counts,
        "faces": diag["faces"],
        "stage_ms": {k: v[0] for k, v in times.items()},
    }
    log_(f"[bench] rungs: {res}")
    return res


def guess_pair(st, scheme, precision, mlp_state, log_, name):
    """One step with the plain and one with the learned guess, both from the
    state st: the flux loop's time (a step without the face dump, whose
    per-face record counter would be timed with it), then, from st again,
    Newton steps per face (mean and 99th percentile, all faces and gated
    faces) and fallbacks of a step with every face dumped."""
    import torch

    from paper_2211_12243_amd import learned, mfm

    out = {}
    n = len(st["x"])
    for guess in (0, 1):
        params = mfm.params_from_dict({"scheme": scheme, "guess": guess}, precision=precision)
        ctx = mfm.Context(params, n)
        if guess:
            mfm.mfm_mlp_attach(ctx, mlp_state)
        ps = mfm.ParticleSet(st, ids=False)
        mfm.mfm_enable_timing(ctx, True)
        mfm.mfm_step(ctx, ps, 1.0)
        torch.cuda.synchronize()
        times = mfm.mfm_kernel_times(ctx)
        mfm.mfm_enable_timing(ctx, False)
        del ps
        ps = mfm.ParticleSet(st, ids=False)
        mfm.mfm_reset_counters(ctx)
        col = learned.Collector(ctx, 24 * n, None, seed=0)
        col.step(ps)
        d = mfm.mfm_diagnostics(ctx)
        r = learned.iteration_stats(col.rows())
        r.update({"flux_ms": times["fluxes"][0], "flux_kernel_ms": times["flux_kernel"][0],
                  "flux_hard_ms": times["flux_hard"][0], "hard_faces": d["hard_faces"],
                  "guess_fallbacks": d["guess_fallback"]})
        out["learned" if guess else "plain"] = r
        del col, ps
        ctx.close()
    log_(f"[bench] {name} {precision} plain vs learned guess: {out}")
    return out


def run_small_configs(args, log_):
    """The shock tube (16^3, MFV, FP64: one full step) and the shear layers
    (64^3, MFV and MFM, FP64 and mixed: 10 steps after 2 warm-up steps):
    ms per step and pair interactions/s per set."""
    import torch

    from paper_2211_12243_amd import mfm
    from paper_2211_12243_amd import workloads as W

    out = {}
    for name, make, scheme, precision, steps in (
            ("sod16_mfv_fp64", lambda: W.sod(n=16, seed=1), "mfv", "fp64", 1),
            ("kh64_mfv_fp64", lambda: W.kh(n=64, seed=2), "mfv", "fp64", 10),
            ("kh64_mfv_mixed", lambda: W.kh(n=64, seed=2), "mfv", "mixed", 10),
            ("kh64_mfm_fp64", lambda: W.kh(n=64, seed=2), "mfm", "fp64", 10),
            ("kh64_mfm_mixed", lambda: W.kh(n=64, seed=2), "mfm", "mixed", 10)):
        st = make()
        n = len(st["x"])
        ctx = mfm.Context(mfm.params_from_dict({"scheme": scheme}, precision=precision), n)
        ps = mfm.ParticleSet(st, ids=False)
        if steps > 1:
            for _ in range(2):
                mfm.mfm_step(ctx, ps, 1.0)
        mfm.mfm_reset_counters(ctx)
        mfm.mfm_enable_timing(ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            mfm.mfm_step(ctx, ps, 1.0)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        times = mfm.mfm_kernel_times(ctx)
        d = mfm.mfm_diagnostics(ctx, ps)
        ctx.close()
        t_pairs = (times["gradients"][0] + times["fluxes"][0]) / 1e3
        out[name] = {"particles": n, "steps": steps, "ms_per_step": ms,
                     "pair_interactions_per_s": (d["grad_pairs"] + d["faces"]) / t_pairs,
                     "stage_ms_per_step": {k: v[0] / steps for k, v in times.items()}}
        log_(f"[bench] {name}: {out[name]}")
    return out


def _state_error(gpu, ref):
    """Per-field difference of two particle states: positions absolute
    (periodic, unit box), velocities against the largest velocity component,
    mass, energy and internal energy against their largest value."""
    import numpy as np

    vscale = max(float(np.abs(ref[k]).max()) for k in ("vx", "vy", "vz"))
    out = {}
    for k in ("x", "y", "z", "vx", "vy", "vz", "m", "E", "U"):
        d = np.abs(gpu[k] - ref[k])
        if k in ("x", "y", "z"):
            out[k] = float(np.minimum(d, 1.0 - d).max())
        elif k in ("vx", "vy", "vz"):
            out[k] = float(d.max() / max(vscale, 1e-300))
        else:
            out[k] = float(d.max() / max(float(np.abs(ref[k]).max()), 1e-300))
    return out


def error_growth(name, st, scheme, precisions, steps, log_):
    """The oracle and one GPU context per precision each step their own copy
    of the set `steps` times (each with its own time step): the largest
    field difference after every step, the per-field differences after the
    last, the largest relative difference of the time steps."""
    import numpy as np
    import torch

    import oracle
    from paper_2211_12243_amd import mfm

    cfg = {"scheme": scheme}
    n = len(st["x"])
    sides = {}
    for prec in precisions:
        ctx = mfm.Context(mfm.params_from_dict(cfg, precision=prec), n)
        sides[prec] = (ctx, mfm.ParticleSet(st))
    ref = {k: np.asarray(st[k], dtype=np.float64).copy() for k in oracle.STATE_KEYS}
    res = {p: {"max_error_per_step": [], "dt_rel_diff_max": 0.0} for p in precisions}
    t0 = time.perf_counter()
    for s in range(steps):
        ref, dt_ref, _ = oracle.step(cfg, ref, 1.0)
        for prec, (ctx, ps) in sides.items():
            dt = mfm.mfm_step(ctx, ps, 1.0)
            torch.cuda.synchronize()
            ids = ps["id"].cpu().numpy()
            gpu = {}
            for k in ("x", "y", "z", "vx", "vy", "vz", "m", "E", "U"):
                a = np.empty(n)
                a[ids] = ps[k].cpu().numpy()
                gpu[k] = a
            e = _state_error(gpu, ref)
            r = res[prec]
            r["max_error_per_step"].append(max(e.values()))
            r["dt_rel_diff_max"] = max(r["dt_rel_diff_max"], abs(dt - dt_ref) / dt_ref)
            r["last_step"] = e
        log_(f"[bench] error growth {name}: step {s + 1} of {steps}, " + ", ".join(
            f"{p} {res[p]['max_error_per_step'][-1]:.2e}" for p in precisions))
    for ctx, _ in sides.values():
        ctx.close()
    out = {"particles": n, "scheme": scheme, "steps": steps,
           "wall_s": time.perf_counter() - t0, **res}
    log_(f"[bench] error growth {name}: {out}")
    return out


def run_clustered(args, st, log_, mlp_state=None):
    """The clustered gas (log-normal density, sigma_ln = 1.5; smoothing lengths
    spread over a factor of about 30): mixed MFM, the first step from the
    initial state (it counts the neighbour lists before planning them) and
    then steady steps."""
    import torch

    from paper_2211_12243_amd import mfm

    n = st["x"].size
    ctx = mfm.Context(mfm.params_from_dict({"scheme": "mfm"}, precision="mixed"), n)
    ps = mfm.ParticleSet(st, ids=False)
    mfm.mfm_enable_timing(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mfm.mfm_step(ctx, ps, 1.0)
    torch.cuda.synchronize()
    first_ms = (time.perf_counter() - t0) * 1e3
    d1 = mfm.mfm_diagnostics(ctx, ps)
    first_times = mfm.mfm_kernel_times(ctx)
    mfm.mfm_enable_timing(ctx, True)  # restarts the stage clocks
    mfm.mfm_reset_counters(ctx)
    K = 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        mfm.mfm_step(ctx, ps, 1.0)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / K * 1e3
    times = mfm.mfm_kernel_times(ctx)
    diag = mfm.mfm_diagnostics(ctx, ps)
    H = ps["H"]
    spread = float((H.max() / H.min()).item())
    now = ps.host(["x", "y", "z", "vx", "vy", "vz", "m", "E", "U", "H"]) if mlp_state else None
    del ps
    ctx.close()
    pair = ({p: guess_pair(now, "mfm", p, mlp_state, log_, "clustered") for p in ("mixed", "fp64")}
            if mlp_state else None)
    del now
    t_pairs = (times["gradients"][0] + times["fluxes"][0]) / 1e3
    res = {
        "workload": f"clustered gas {args.clustered}^3 (log-normal, sigma_ln 1.5, vrms 10 c_s), "
                    "MFM mixed",
        "particles": n,
        "first_step_ms": first_ms,
        "first_step_rebuilds": d1["cell_rebuilds"],
        "first_step_stage_ms": {k: v[0] for k, v in first_times.items()},
        "ms_per_step": ms,
        "steps": K,
        "pair_interactions_per_s": (diag["grad_pairs"] + diag["faces"]) / t_pairs,
        "stage_ms_per_step": {k: v[0] / K for k, v in times.items()},
        "pairs_per_step": {"gradient": diag["grad_pairs"] / K, "flux_faces": diag["faces"] / K},
        "list_retries": diag["list_overflow"],
        "h_spread": spread,
        "vacuum_faces_per_step": diag["vacuum"] / K,
        "guess": pair,
    }
    log_(f"[bench] clustered: {res}")
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the library "
              "runs on a single GPU and has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2211_12243_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    variants = [v for v in args.variants.split(",") if v]
    for v in variants:
        if v not in VARIANTS:
            print(f"unknown variant {v}", file=sys.stderr)
            sys.exit(2)
    if args.headline not in variants:
        args.headline = variants[-1]

    def log_(m):
        log(m, args)

    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log_(f"[bench] copy probe: {args.copy_probe_mib} MiB read and written once")
        del src, dst
    t = time.perf_counter()
    st = W.sedov(n=args.n, seed=3)
    N = len(st["x"])
    log_(f"[bench] sedov n={args.n}^3 ({N} particles) made in {time.perf_counter() - t:.1f}s")
    c4 = None
    if args.clustered > 0 or "mixed_learned" in variants:
        t = time.perf_counter()
        nc = args.clustered if args.clustered > 0 else 64
        c4 = W.clustered(n=nc, seed=4)
        log_(f"[bench] clustered n={nc}^3 ({c4['x'].size} particles) made in "
             f"{time.perf_counter() - t:.1f}s")
    mlp_state, train_info = (None, None)
    if "mixed_learned" in variants:
        mlp_state, train_info = train_guess(args, c4, log_)
    res = {v: run_variant(args, st, v, mlp_state, log_) for v in variants}
    rungs = (run_rungs(args, st, res["fp64"]["ms_per_step"], log_)
             if args.rung_base > 0 and "fp64" in res else None)
    clustered = run_clustered(args, c4, log_, mlp_state) if args.clustered > 0 else None
    del c4
    small = run_small_configs(args, log_) if args.small_configs else None
    h = res[args.headline]
    out = {
        "metric": "pair interactions/s (grad+flux) & hydro-step ms, 2.1M Sedov, mixed vs FP64",
        "value": h["value"],
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.headline == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"sedov {args.n}^3 MFM blast (lattice + 0.1 jitter, P=1e-6, "
                               f"E=1 in central 33)", "particles": N, "scheme": args.scheme,
                   "variant": args.headline, "n_ngb": 32, "gamma": 5.0 / 3.0},
        "roofline": h["roofline"],
        "variants": {v: {k: r[k] for k in ("value", "ms_per_step", "stage_ms_per_step",
                                           "newton_iters_per_face", "fp64_pass_faces_frac",
                                           "guess_fallback_frac", "newton_after",
                                           "kernels")}
                     for v, r in res.items()},
        "pairs_per_step": h["pairs_per_step"],
        "guess_training": train_info,
        "individual_steps": rungs,
        "clustered": clustered,
        "small_configs": small,
    }
    if not args.no_cpu_baseline:
        fields = {v: step1_fields(args, st, v) for v in ("fp64", "mixed") if v in variants}
        log_("[bench] timing the CPU oracle on one step of the same set")
        out["cpu_baseline"] = cpu_baseline(st, args.scheme, fields)
        if args.error_growth:
            from paper_2211_12243_amd import workloads as W

            both = ("fp64", "mixed")
            out["error_growth"] = {
                "kh64_mfv": error_growth("kh64_mfv", W.kh(n=64, seed=2), "mfv", both, 10, log_),
                "kh64_mfm": error_growth("kh64_mfm", W.kh(n=64, seed=2), "mfm", both, 10, log_),
                f"sedov{args.n}_mfm": error_growth(f"sedov{args.n}_mfm", st, "mfm", both, 20,
                                                   log_)}
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
