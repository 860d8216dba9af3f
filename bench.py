"""Benchmark: MFM hydro steps of the 2.1M-particle Sedov blast on one MI355X.

Workload: 128^3 particles, lattice + 0.1-spacing jitter, rho = 1, P = 1e-6, unit
energy deposited kernel-weighted in the central 33 particles, gamma = 5/3,
N_NGB = 32, MFM scheme.  Each timed step is one mfm_step: cell build (sort),
neighbour search, density / smoothing-length loop, gradients + time step,
fluxes, update -- the whole hot path, inputs resident in HBM.

Variants, each from the same initial set with the same warm-up:
  fp64           all pair arithmetic in FP64;
  mixed          FP32 pair arithmetic, FP64 accumulators and checks;
  mixed_learned  mixed, with the Riemann iteration started from the guess
                 network (trained first, on faces dumped from other sets).
The reported value is the headline variant's (default mixed: FP32 pair
arithmetic with FP64 accumulators, 1e-5 parity with the FP64 oracle); every
variant's rate and stage times are in "variants".

Metric: pair interactions per second over the gradient and flux loops,
(gradient pairs + flux faces) / (t_gradients + t_fluxes), with the loop times
from HIP events the library records on its own stream; ms per full step is
reported beside it.

The JSON line also carries
  roofline     -- the dominant kernel (the flux loop) against the vector ALU
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


VARIANTS = ("fp64", "mixed", "mixed_learned")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=128, help="particles per axis")
    ap.add_argument("--variants", default=",".join(VARIANTS),
                    help="comma-separated subset of " + ", ".join(VARIANTS))
    ap.add_argument("--headline", default="mixed", choices=VARIANTS,
                    help="variant whose rate is the reported value")
    ap.add_argument("--scheme", default="mfm", choices=["mfm", "mfv"])
    ap.add_argument("--train-steps", type=int, default=800)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy a buffer of this many MiB on the device (a kernel of "
                         "known traffic, to calibrate hardware byte counters)")
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


def train_guess(args, log_):
    """Train the guess network on faces the plain mixed solver dumps from
    other sets than the timed one (Sedov 64^3 with another seed, after two
    steps, and the 64^3 Kelvin-Helmholtz layers); returns (state, info)."""
    import numpy as np
    import torch

    from paper_2211_12243_amd import mfm
    from paper_2211_12243_amd import workloads as W

    t0 = time.perf_counter()
    parts = []
    for name, st, skip in (("sedov64", W.sedov(n=64, seed=17), 2), ("kh64", W.kh(n=64, seed=2), 0)):
        params = mfm.params_from_dict({"scheme": args.scheme}, precision="mixed")
        ctx = mfm.Context(params, len(st["x"]))
        ps = mfm.ParticleSet(st, ids=False)
        for _ in range(skip):
            mfm.mfm_step(ctx, ps, 1.0)
        rec = torch.empty((4_000_000, mfm.DUMP_STRIDE), dtype=torch.float32, device="cuda")
        mfm.mfm_face_dump(ctx, rec)
        mfm.mfm_step(ctx, ps, 1.0)
        cnt = mfm.mfm_face_dump_count(ctx)
        mfm.mfm_face_dump(ctx, None)
        sel = rec[:cnt][mfm.guess_gate(rec[:cnt])]
        parts.append(sel)
        log_(f"[bench] dumped {cnt} faces from {name}, {sel.shape[0]} pass the guess gate")
        ctx.close()
    rows = torch.cat(parts)
    r = rows[:, :7].double()
    mean, std = r.mean(0).cpu().numpy(), r.std(0).cpu().numpy()
    norm = np.zeros(16, dtype=np.float32)
    norm[:6], norm[6:12] = mean[:6], np.maximum(std[:6], 1e-6)
    norm[12], norm[13] = mean[6], max(std[6], 1e-6)
    rng = np.random.default_rng(0)
    p0 = np.zeros(mfm.mfm_mlp_param_count(), dtype=np.float32)
    lay = mfm.mlp_param_layout()
    for name, (off, shp) in lay.items():
        if name.startswith("W") or name == "w4":
            fan = 6 if name == "W1" else 64
            w = rng.normal(0, np.sqrt((1.0 if name == "w4" else 2.0) / fan), shp)
            if name == "W1":
                w[6:] = 0.0
            p0[off:off + w.size] = w.ravel()
    stt = mfm.MLPState(p0, norm)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g = torch.Generator(device="cuda").manual_seed(0)
    n = rows.shape[0]
    losses = []
    for it in range(args.train_steps):
        lr = 3e-3 if it < 0.7 * args.train_steps else 1e-3
        idx = torch.randint(0, n, (16384,), device="cuda", generator=g)
        want = it in (0, args.train_steps - 1)
        loss = mfm.mfm_mlp_train_step(stt, rows[idx], lr, want_loss=want)
        if want:
            losses.append(loss)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = {"faces": int(n), "dump_s": t1 - t0, "train_s": t2 - t1, "steps": args.train_steps,
            "batch": 16384, "loss_first": losses[0], "loss_last": losses[-1]}
    log_(f"[bench] trained guess network: {info}")
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
    ctx.close()
    K = args.steps
    t_grad = times["gradients"][0] / 1e3
    t_flux = times["fluxes"][0] / 1e3
    pairs = diag["grad_pairs"] + diag["faces"]
    n_launch = max(times["fluxes"][1], 1)
    mean_s = t_flux / n_launch
    flops_launch = (diag["faces"] * FLOPS_FACE[args.scheme]
                    + diag["riemann_iters"] * FLOPS_NEWTON_ITER) / n_launch
    peak = PEAK_FP64_TFLOPS if precision == "fp64" else PEAK_FP32_TFLOPS
    achieved = flops_launch / mean_s / 1e12
    res = {
        "value": pairs / (t_grad + t_flux),
        "ms_per_step": (t1 - t0) / K * 1e3,
        "stage_ms_per_step": {k: v[0] / K for k, v in times.items()},
        "pairs_per_step": {"gradient": diag["grad_pairs"] / K, "flux_faces": diag["faces"] / K},
        "newton_iters_per_face": diag["riemann_iters"] / max(diag["faces"], 1),
        "guess_fallback_frac": diag["guess_fallback"] / max(diag["faces"], 1),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": flux_traffic(variant),
                     "kernel": "fluxes_k",
                     "mean_launch_ms": mean_s * 1e3, "flops_per_launch": flops_launch},
        "conserved_after": {k: diag[k] for k in ("mass", "px", "py", "pz", "energy")},
    }
    log_(f"[bench] {variant}: {res}")
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
    mlp_state, train_info = (None, None)
    if "mixed_learned" in variants:
        mlp_state, train_info = train_guess(args, log_)
    res = {v: run_variant(args, st, v, mlp_state, log_) for v in variants}
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
                                           "newton_iters_per_face", "guess_fallback_frac")}
                     for v, r in res.items()},
        "pairs_per_step": h["pairs_per_step"],
        "guess_training": train_info,
    }
    if not args.no_cpu_baseline:
        log_("[bench] timing the CPU oracle on one step of the same set")
        out["cpu_baseline"] = cpu_baseline(st, args.scheme)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
