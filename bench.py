#!/usr/bin/env python3
"""Coupled-step throughput of the electroconvection time step on one MI355X.

Workload (the bandwidth configuration): nx = ny = 4096, FP32-deviation
storage (collision arithmetic in FP64, the mode that meets the 1e-5 parity
gate; --precision fp32 for FP32 arithmetic), T = 500, C = 10, M = 10, Fe = 4000, Lambda = 1/4, Lambda_g = 1e-6,
tau+ = 0.8, hydrostatic initial state with seeded relative charge noise 1e-4.
A step is one pass of the whole coupled path: charge gather and forward
x-transform, x-mean Poisson mode, per-wavenumber solves, inverse transform,
fused collide-stream of both lattices.  Inputs are resident in HBM before the
timed region starts.

Prints one JSON line:
  value          coupled-step MLUPS (lattice-node updates per second / 1e6)
  roofline       the collide-stream kernel (the dominant one): algorithmic
                 bytes per launch (148 B/node FP32, 296 FP64) over its average
                 launch time from HIP events recorded on its stream during the
                 timed region, against 8 TB/s
  step_roofline  the whole step against the HBM roofline of its algorithmic
                 bytes (176 B/node FP32)
  cpu_baseline   the FP64 oracle on the host (same grid, two timed steps)
  serve          the served stream: Poisson arrivals at 50 requests/s, ny in
                 {64, 128, 256, 512} with weights 0.4 / 0.3 / 0.2 / 0.1, nx =
                 smallest 5-smooth >= round(1.22 ny), T uniform in [120, 400],
                 C in {1, 10, 100}, FP32 storage, 5000 steps per request,
                 admission by workspace footprint; 2000 requests of which the
                 first 200 warm up; p50 / p99 latency from arrival to final
                 fields, runs/s, longest admission queue
  serve_admission_bound  the same stream on a 0.25 GB workspace, where
                 admission by footprint binds (requests queue for memory)
  sweep          the batched T sweep: 64 instances, ny uniform in 64..256,
                 nx = smallest 5-smooth >= round(1.22 ny), T uniform in
                 [100, 250], C = 10, M = 10, FP32 storage, 20000 steps each,
                 autotuned launch shapes, one batch (captured HIP graphs),
                 against the same instances run one at a time through
                 lbm_ec_step (timed over 1000 steps each, scaled to 20000);
                 per instance the ionic times the run covers and the slope of
                 ln A1 with its R^2, a growth rate only where the run covers
                 at least one ionic time (a transient slope otherwise)
  hysteresis     Ne_0 = I / I_0 on both branches of section V.2 in one batch
                 on a 61 x 50 channel (C = 10, M = 10, Fe = 4000, FP32
                 storage): runs from rest at T = 155, 160, 165; one run whose
                 vortices form at T = 200 (12 ionic times), then continued at
                 T = 150, 120, 110, 108, 106, 104 (6 ionic times each);
                 brackets of T_c and T_f (paper: 163.4 and 108.7), run time
"""

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COLLIDE_BYTES_PER_NODE = {"fp32": 152, "fp32_f64math": 152, "fp64": 304}
STEP_BYTES_PER_NODE = {"fp32": 176, "fp32_f64math": 176, "fp64": 352}
WORKLOAD = dict(T=500.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8, Lambda=0.25, Lambda_g=1e-6,
                noise_amp=1e-4, seed=181205711)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("ec_kernels.hip", "ec_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1812_05711_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(nx, ny, precision):
    """HBM bytes per collide launch from the committed counter summary
    (profiles/collide_<nx>x<ny>_<precision>_hbm_counters.md), if it was taken
    on the current kernel source and the same workload; else None."""
    path = os.path.join(ROOT, "profiles", f"collide_{nx}x{ny}_{precision}_hbm_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", "|", " ")):
            k, _, v = line.partition(":")
            vals[k.strip()] = v.strip()
    try:
        ok = (vals.get("source_hash") == kernel_source_hash() and int(vals.get("nx", -1)) == nx
              and int(vals.get("ny", -1)) == ny and vals.get("precision") == precision)
        return float(vals["traffic_bytes_per_launch"]) if ok else None
    except (KeyError, ValueError):
        return None


CPU_SNIPPET = r"""
import json, os, sys, time
sys.path.insert(0, {root!r})
from oracle import Oracle, Params
p = Params(nx={nx}, ny={ny}, **{kw!r})
o = Oracle(p)
o.step(1)
t = time.perf_counter()
o.step({steps})
dt = time.perf_counter() - t
print(json.dumps(dict(seconds=dt, steps={steps})))
"""


def cpu_baseline(nx, ny, steps=3):
    """The oracle on a bounded sample of the workload: the same row length and
    parameters on a slab of at most 2048 rows (its cost per node does not
    depend on the row count), `steps` timed steps after one untimed."""
    ny = min(ny, 2048)
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    code = CPU_SNIPPET.format(root=ROOT, nx=nx, ny=ny, kw=WORKLOAD, steps=steps)
    log(f"cpu baseline: oracle at {nx}x{ny}, {steps} timed steps, 1 thread")
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=900)
    if res.returncode != 0:
        log("cpu baseline failed: " + res.stderr[-500:])
        return None
    r = json.loads(res.stdout.strip().splitlines()[-1])
    mlups = nx * ny * r["steps"] / r["seconds"] / 1e6
    return {"value": mlups, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"FP64 NumPy oracle on a {nx}x{ny} slab of the workload (same row length and parameters), "
                      f"{r['steps']} steps after one untimed step ({r['seconds']:.1f} s), single thread"}


def sweep_section(steps, plain_steps):
    import numpy as np

    from paper_1812_05711_amd import sweep

    cfgs = sweep.sweep_configs()
    nodes = sum(c["nx"] * c["ny"] for c in cfgs)
    log(f"sweep: {len(cfgs)} instances, {nodes} nodes, {steps} steps, batched")
    r = sweep.run_batched(cfgs, steps)
    log(f"sweep: batched {r['seconds']:.2f} s; plain, {plain_steps} steps each")
    tp = sweep.run_plain(cfgs, plain_steps) * steps / plain_steps
    T = [c["T"] for c in cfgs]
    fits = r["fits"]
    order = np.argsort(T)
    # a rate is reported as a number only where the run covers at least one
    # ionic time; shorter runs give the early transient, reported with the fit
    # quality but not as a growth rate
    rates = []
    for i in order:
        f = fits[i]
        rates.append({"T": round(T[i], 2), "ny": cfgs[i]["ny"], "ionic_times": round(f["span"], 3),
                      "growth_rate": None if f["transient"] else round(f["rate"], 4),
                      "transient_slope": round(f["rate"], 4) if f["transient"] else None,
                      "fit_r2": round(f["r2"], 4)})
    return {"instances": len(cfgs), "steps": steps, "nodes": nodes,
            "batched_runs_per_s": len(cfgs) / r["seconds"], "plain_runs_per_s": len(cfgs) / tp,
            "speedup": tp / r["seconds"], "batched_seconds": r["seconds"], "plain_seconds": tp,
            "batched_mlups": nodes * steps / r["seconds"] / 1e6,
            "us_per_step": r["seconds"] / steps * 1e6,
            "plain_sample": f"{plain_steps} steps per instance, scaled to {steps}",
            "tuning": list(r["tuning"]) if r["tuning"] else None,
            "instances_over_one_ionic_time": sum(1 for f in fits if not f["transient"]),
            "growth_by_T": rates}


def serve_section(n, warmup, budget_gb, tag="serve"):
    from paper_1812_05711_amd.serve import BatchBackend, make_requests, serve

    from paper_1812_05711_amd import autotune

    reqs = make_requests(n, rate=50.0, steps=5000)
    # launch shapes tuned on a sample of the stream's mix (before the clock starts)
    tuning = autotune.tune_batch([r["params"] for r in reqs[:48]])
    log(f"{tag}: {n} requests at 50/s, budget {budget_gb} GB, launch shapes {tuning}")
    be = BatchBackend(int(budget_gb * (1 << 30)), max_slots=512, tuning=tuning)
    records, summary = serve(reqs, be, chunk=100, warmup=warmup, max_wall=900.0)
    be.close()
    summary.update({"rate_per_s": 50.0, "steps_per_request": 5000, "warmup_requests": warmup,
                    "budget_bytes": int(budget_gb * (1 << 30)), "chunk_steps": 100, "tuning": list(tuning)})
    summary["refused"] = len(summary["refused"])
    log(f"{tag}: p50 {summary['p50_s']:.3f} s, p99 {summary['p99_s']:.3f} s, {summary['runs_per_s']:.1f} runs/s, "
        f"longest queue {summary['max_queue']}")
    return summary


def hysteresis_section():
    from paper_1812_05711_amd import hysteresis

    rise, fall = (155.0, 160.0, 165.0), (200.0, 150.0, 120.0, 110.0, 108.0, 106.0, 104.0)
    log(f"hysteresis: 61 x 50, rising {rise}, falling {fall}")
    r = hysteresis.run(nx=61, ny=50, T_rise=rise, T_fall=fall, start_t0=12.0, dwell_t0=6.0,
                       progress=lambda m: log("hysteresis: " + m))
    log(f"hysteresis: T_c in {r['T_c_bracket']}, T_f in {r['T_f_bracket']}, {r['seconds']:.1f} s")
    keep = ("grid", "steps", "slots", "seconds", "us_per_step", "mlups", "healthy", "rising", "falling",
            "T_c_bracket", "T_f_bracket", "start_t0", "dwell_t0", "tuning")
    out = {k: r[k] for k in keep}
    out["rising"] = [[T, round(v, 5)] for T, v in r["rising"]]
    out["falling"] = [[T, round(v, 5)] for T, v in r["falling"]]
    out["paper"] = {"T_c": 163.4, "T_f": 108.7}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--nx", type=int, default=4096)
    ap.add_argument("--ny", type=int, default=4096)
    ap.add_argument("--precision", default="fp32_f64math", choices=["fp32", "fp32_f64math", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-hysteresis", action="store_true")
    ap.add_argument("--T", type=float, default=WORKLOAD["T"], help="electric Rayleigh number")
    ap.add_argument("--noise-amp", type=float, default=WORKLOAD["noise_amp"], help="relative charge noise")
    ap.add_argument("--y-solver", default="tridiagonal", choices=["tridiagonal", "spectral"],
                    help="y solve of the m >= 1 modes (spectral: the odd-extension route of Eq. 21-25)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
    ap.add_argument("--serve-bound-budget-gb", type=float, default=0.25,
                    help="budget of the second serve leg, small enough that admission by footprint binds "
                         "(0: no second leg)")
    ap.add_argument("--sweep-steps", type=int, default=20000)
    ap.add_argument("--sweep-plain-steps", type=int, default=1000)
    args = ap.parse_args()

    WORKLOAD.update(T=args.T, noise_amp=args.noise_amp)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the time step runs on a single GPU: independent instances would shard across GPUs by "
              "footprint, one large instance in y-slabs with one-row halo exchanges)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1812_05711_amd.lbm_ec import Simulation

    nx, ny = args.nx, args.ny
    log(f"create {nx}x{ny} {args.precision}")
    sim = Simulation(device="cuda:0", nx=nx, ny=ny, precision=args.precision, **WORKLOAD)
    sim.set_y_solver(args.y_solver)
    torch.cuda.synchronize()
    tuning = None
    if not args.no_tune:
        from paper_1812_05711_amd import autotune

        tuning, t_ms = autotune.tune_single(sim, steps=8)
        log(f"tuned launch shapes {tuning} ({t_ms:.3f} ms/step while tuning)")
    log(f"warmup {args.warmup} steps")
    sim.step(args.warmup)
    torch.cuda.synchronize()

    # the timed region times the dominant kernel (the collide) with HIP events
    # on the library's stream; each event pair costs a few microseconds, so the
    # other kernel classes are timed in a separate pass after it
    log(f"timed {args.steps} steps")
    sim.profile_begin(["collide"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sim.profile_end()
    seconds = t1 - t0
    st, healthy = sim.stats()
    log(f"done: {seconds * 1e3 / args.steps:.3f} ms/step, healthy={healthy}")
    kpass = max(10, min(100, args.steps))
    sim.profile_begin()
    sim.step(kpass)
    prof_all = sim.profile_end()

    nodes = nx * ny
    mlups = nodes * args.steps / seconds / 1e6
    kernels = {k: {"avg_us": (ms / n * 1e3) if n else None, "launches": n} for k, (ms, n) in prof_all.items()}
    kernels["pass"] = f"{kpass} steps after the timed region, every kernel class timed"
    c_ms, c_n = prof["collide"]
    c_avg_s = c_ms / c_n / 1e3
    c_bytes = COLLIDE_BYTES_PER_NODE[args.precision] * nodes
    achieved = c_bytes / c_avg_s / 1e9
    traffic = traffic_from_profiles(nx, ny, args.precision)
    roofline_mlups = HBM_PEAK_GBS * 1e9 / STEP_BYTES_PER_NODE[args.precision] / 1e6

    out = {
        "metric": "coupled-step MLUPS",
        "value": mlups,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": seconds * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp32_f64math": "f32 storage / f64 collision", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"coupled TRT-LBM / FFT-Poisson electroconvection step, {nx}x{ny}, "
                               f"{'FP64' if args.precision == 'fp64' else 'FP32-deviation'} storage, "
                               f"T={args.T:g} C=10 M=10 Fe=4000, seeded charge noise {args.noise_amp:g}",
                   "nx": nx, "ny": ny, "precision": args.precision, "y_solver": args.y_solver},
        "roofline": {"bound": "hbm", "kernel": "collide-stream", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_gbs": (traffic / c_avg_s / 1e9) if traffic else None,
                     "algorithmic_bytes_per_launch": c_bytes, "avg_launch_us": c_avg_s * 1e6},
        "step_roofline": {"algorithmic_bytes_per_node": STEP_BYTES_PER_NODE[args.precision],
                          "roofline_mlups": roofline_mlups, "frac": mlups / roofline_mlups},
        "kernels": kernels,
        "tuning": list(tuning) if tuning else None,
        "healthy": bool(healthy),
    }
    del sim
    torch.cuda.empty_cache()
    out["sweep"] = None if args.no_sweep else sweep_section(args.sweep_steps, args.sweep_plain_steps)
    out["serve"] = None if args.no_serve else serve_section(args.serve_requests, args.serve_warmup,
                                                            args.serve_budget_gb)
    out["serve_admission_bound"] = (None if args.no_serve or args.serve_bound_budget_gb <= 0 else
                                    serve_section(args.serve_requests, args.serve_warmup,
                                                  args.serve_bound_budget_gb, tag="serve (bound)"))
    out["hysteresis"] = None if args.no_hysteresis else hysteresis_section()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(nx, ny)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
