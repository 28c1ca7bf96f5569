#!/usr/bin/env python3
"""Coupled-step throughput of the electroconvection time step on one MI355X.

Workload (the bandwidth configuration): nx = ny = 4096, FP32-deviation
storage, T = 500, C = 10, M = 10, Fe = 4000, Lambda = 1/4, Lambda_g = 1e-6,
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
COLLIDE_BYTES_PER_NODE = {"fp32": 148, "fp32_f64math": 148, "fp64": 296}
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
    """HBM bytes per collide launch from the committed counter summary, if it
    was taken on the current kernel source and the same workload."""
    path = os.path.join(ROOT, "profiles", "collide_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except Exception:
        return None
    if t.get("source_hash") != kernel_source_hash() or t.get("nx") != nx or t.get("ny") != ny \
            or t.get("precision") != precision:
        return None
    return t.get("hbm_bytes_per_launch")


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


def cpu_baseline(nx, ny, steps=2):
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
            "sample": f"FP64 NumPy oracle, full {nx}x{ny} grid, {r['steps']} steps after one untimed step "
                      f"({r['seconds']:.1f} s), single thread"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--nx", type=int, default=4096)
    ap.add_argument("--ny", type=int, default=4096)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp32_f64math", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the time step runs on a single GPU; see DESIGN.md for how it would shard)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1812_05711_amd.lbm_ec import Simulation

    nx, ny = args.nx, args.ny
    log(f"create {nx}x{ny} {args.precision}")
    sim = Simulation(device="cuda:0", nx=nx, ny=ny, precision=args.precision, **WORKLOAD)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} steps")
    sim.step(args.warmup)
    torch.cuda.synchronize()

    log(f"timed {args.steps} steps")
    sim.profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sim.profile_end()
    seconds = t1 - t0
    st, healthy = sim.stats()
    log(f"done: {seconds * 1e3 / args.steps:.3f} ms/step, healthy={healthy}")

    nodes = nx * ny
    mlups = nodes * args.steps / seconds / 1e6
    kernels = {k: {"avg_us": (ms / n * 1e3) if n else None, "launches": n} for k, (ms, n) in prof.items()}
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
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"coupled TRT-LBM / FFT-Poisson electroconvection step, {nx}x{ny}, "
                               f"{'FP32-deviation' if args.precision == 'fp32' else 'FP64'} storage, "
                               "T=500 C=10 M=10 Fe=4000, seeded charge noise 1e-4",
                   "nx": nx, "ny": ny, "precision": args.precision},
        "roofline": {"bound": "hbm", "kernel": "collide-stream", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": c_bytes, "avg_launch_us": c_avg_s * 1e6},
        "step_roofline": {"algorithmic_bytes_per_node": STEP_BYTES_PER_NODE[args.precision],
                          "roofline_mlups": roofline_mlups, "frac": mlups / roofline_mlups},
        "kernels": kernels,
        "healthy": bool(healthy),
    }
    del sim
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(nx, ny)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
