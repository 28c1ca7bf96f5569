"""T sweeps for locating the electroconvective threshold: many uneven
instances advanced as one batch (paper section V.2: the threshold T_c is
where perturbations stop decaying).

Each instance is a channel of ny rows with nx the smallest 5-smooth length
not below round(1.22 ny) (the aspect ratio 1.22 of the paper's domain), its
own T and seed; all share C, M, Fe and the precision.  The growth rate of an
instance is the least-squares slope of ln A1 against t / t0 (A1 the
amplitude of the first x mode of u_y, the largest over the rows; t0 = H^2 / K,
the ionic time) over the second half of its run, from the rows the batch
records every `emit_every` steps.  (rms u_y would mix in the other modes,
which decay at their own rates.)
"""

import time

import numpy as np

from . import autotune
from .lbm_ec import Batch, Simulation, batch_workspace_bytes, make_params
from .workloads import five_smooth_at_least, sweep_configs  # noqa: F401 (the sweep's instance list)


def ionic_time(cfg):
    nu = (cfg["tau_plus"] - 0.5) / 3.0
    K = nu * cfg["T"] / cfg["M"] ** 2
    return cfg["ny"] ** 2 / K


def growth_rate(history, t0, col=4):
    """Slope of ln(history[:, col]) versus t / t0 over the second half of the
    rows (col 4: the first x mode of u_y)."""
    return growth_fit(history, t0, col)["rate"]


def growth_fit(history, t0, col=4):
    """The growth-rate fit of growth_rate with its quality: rate (per ionic
    time), r2 (coefficient of determination of the straight line through
    ln A over the fitted half), span (ionic times the whole run covers) and
    transient (True when the run covers less than one ionic time, so that
    the rate describes the early transient rather than the linear growth or
    decay that locates T_c)."""
    rows = history[history[:, 0] > 0]
    if len(rows) < 4:
        return dict(rate=float("nan"), r2=float("nan"), span=0.0, transient=True)
    rows = rows[np.argsort(rows[:, 0])]
    h = len(rows) // 2
    t = rows[h:, 0] / t0
    a = np.log(np.maximum(rows[h:, col], 1e-300))
    p = np.polyfit(t, a, 1)
    res = a - np.polyval(p, t)
    ss = float(np.sum((a - a.mean()) ** 2))
    r2 = 1.0 - float(np.sum(res ** 2)) / ss if ss > 0 else 1.0
    span = float(rows[-1, 0] / t0)
    return dict(rate=float(p[0]), r2=r2, span=span, transient=span < 1.0)


def make_batch(configs, steps, emit_every=100, device="cuda:0", tuning=None):
    hist_rows = steps // max(emit_every, 1) + 2
    params = [make_params(**c) for c in configs]
    ws = batch_workspace_bytes(params, len(configs), hist_rows) + (1 << 20)
    b = Batch(len(configs), ws, precision=configs[0]["precision"], emit_every=emit_every, hist_rows=hist_rows,
              device=device)
    if tuning is not None:
        b.set_tuning(*tuning)
    slots = [b.admit(steps, **c) for c in configs]
    if None in slots:
        raise RuntimeError("batch workspace too small")
    return b, slots


def run_batched(configs, steps, emit_every=100, device="cuda:0", tune=True, progress=None, chunk=None):
    """Advances every instance `steps` steps as one batch.  Returns the wall
    time of the stepping (creation excluded), the growth rates, the tuning.
    With `progress`, the steps go in chunks of `chunk` and each chunk ends
    with a call progress(message)."""
    tuning = autotune.tune_batch(configs, device=device) if tune else None
    b, slots = make_batch(configs, steps, emit_every, device, tuning)
    b.stream.synchronize()
    t = time.perf_counter()
    if progress is None:
        b.step(steps)
    else:
        done, chunk = 0, max(1, chunk or steps)
        while done < steps:
            n = min(chunk, steps - done)
            b.step(n)
            b.stream.synchronize()
            done += n
            progress(f"{done} of {steps} steps, {time.perf_counter() - t:.1f} s")
    b.stream.synchronize()
    dt = time.perf_counter() - t
    done = b.poll()
    assert sorted(done) == sorted(slots)
    fits = [growth_fit(b.history(s), ionic_time(c)) for s, c in zip(slots, configs)]
    b.close()
    return dict(seconds=dt, growth=[f["rate"] for f in fits], fits=fits, tuning=tuning)


def run_plain(configs, steps, device="cuda:0"):
    """Each instance alone through lbm_ec_step, one after another.  Returns
    the summed stepping time (creation excluded)."""
    import torch

    total = 0.0
    for c in configs:
        sim = Simulation(device=device, **c)
        torch.cuda.synchronize()
        t = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        total += time.perf_counter() - t
        sim.close()
    return total


def threshold_configs(nx, ny, Ts, precision="fp64", C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8, Lambda=0.25,
                      Lambda_g=1e-6, seed=181205711):
    """The threshold problem of section V.2 at one grid: the Eq. 29
    perturbation on the hydrostatic rows, one instance per T."""
    return [dict(nx=nx, ny=ny, T=float(T), C=C, M=M, Fe=Fe, tau_plus=tau_plus, Lambda=Lambda, Lambda_g=Lambda_g,
                 init_mode="eq29", noise_amp=0.0, seed=seed, instance_id=i, precision=precision)
            for i, T in enumerate(Ts)]


def zero_crossing(Ts, rates):
    """T where the growth rate changes sign, by linear interpolation between
    the neighbouring T values that bracket it (None when none do)."""
    pairs = sorted(zip(Ts, rates))
    for (t0, r0), (t1, r1) in zip(pairs[:-1], pairs[1:]):
        if r0 < 0.0 <= r1:
            return t0 + (t1 - t0) * (-r0) / (r1 - r0)
    return None


def main(argv=None):
    """Command line: runs the seeded T sweep as one batch and prints the
    step time, the throughput and the growth rate of each instance."""
    import argparse

    ap = argparse.ArgumentParser(description="batched T sweep (one batch of uneven instances)")
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--emit-every", type=int, default=100)
    ap.add_argument("--precision", default="fp32_f64math", choices=["fp64", "fp32", "fp32_f64math"])
    ap.add_argument("--tuning", default=None, help="fft_threads,collide_bx,collide_by[,collide_tw] (default: autotuned)")
    ap.add_argument("--threshold", default=None,
                    help="NXxNY: instead of the seeded sweep, the Eq. 29 threshold problem at this grid for the "
                         "T values of --T; prints the growth rates and their zero crossing")
    ap.add_argument("--T", default="160,162,164,166", help="T values of --threshold (comma separated)")
    ap.add_argument("--Lambda", type=float, default=0.25,
                    help="fluid TRT parameter of Eq. 17 for --threshold (the paper's study uses 1/12)")
    ap.add_argument("--tau-plus", type=float, default=0.8, help="fluid tau+ for --threshold")
    args = ap.parse_args(argv)
    if args.threshold:
        nx, ny = (int(v) for v in args.threshold.lower().split("x"))
        Ts = [float(v) for v in args.T.split(",")]
        cfgs = threshold_configs(nx, ny, Ts, precision=args.precision, Lambda=args.Lambda, tau_plus=args.tau_plus)
        import sys

        r = run_batched(cfgs, args.steps, emit_every=args.emit_every, tune=args.tuning is None,
                        progress=lambda m: print(m, file=sys.stderr, flush=True), chunk=200000)
        for T, g in zip(Ts, r["growth"]):
            print(f"T {T:8.3f}  growth rate {g:+.5f} per ionic time", flush=True)
        print(f"zero crossing: T_c = {zero_crossing(Ts, r['growth'])}  ({args.steps} steps, "
              f"{r['seconds']:.1f} s)", flush=True)
        return
    cfgs = sweep_configs(n=args.instances, precision=args.precision)
    tuning = (tuple(int(v) for v in args.tuning.split(",")) if args.tuning
              else autotune.tune_batch(cfgs))
    b, slots = make_batch(cfgs, args.steps, emit_every=args.emit_every, tuning=tuning)
    b.stream.synchronize()
    t = time.perf_counter()
    b.step(args.steps)
    b.stream.synchronize()
    dt = time.perf_counter() - t
    assert sorted(b.poll()) == sorted(slots)
    nodes = sum(c["nx"] * c["ny"] for c in cfgs)
    print(f"{len(cfgs)} instances, {nodes} nodes, {args.steps} steps, tuning {tuning}: "
          f"{dt / args.steps * 1e6:.1f} us per step, {nodes * args.steps / dt / 1e6:.0f} MLUPS", flush=True)
    for s, c in zip(slots, cfgs):
        fit = growth_fit(b.history(s), ionic_time(c))
        kind = "transient slope" if fit["transient"] else "growth rate"
        print(f"  ny {c['ny']:4d} nx {c['nx']:4d} T {c['T']:7.2f} {kind} {fit['rate']:+.4f} per ionic time "
              f"(the run covers {fit['span']:.3f} ionic times; r2 of the fit {fit['r2']:.4f})")
    b.close()


if __name__ == "__main__":
    main()
