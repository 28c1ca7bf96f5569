"""Hysteresis of electroconvection in T (paper section V.2, Fig. 3).

The electric Nusselt number Ne_0 = I / I_0 compares the cathode (collector)
current I of a run with the current I_0 of the hydrostatic solution at the
same parameters.  Two branches, every run a slot of one batch:

  rising:  one run per T, from the hydrostatic state with the Eq. 29
           perturbation.  Below T_c the perturbation decays (Ne_0 -> 1);
           above it the vortices grow to a steady state (Ne_0 > 1).
  falling: one run started at the highest T grows its vortices; T is then
           lowered stage by stage (lbm_ec_batch_set_T, the continuation of
           the paper).  The vortices persist below T_c, down to T_f, where
           the run returns to the hydrostatic state.

I_0 comes from companion slots: the same parameters on a channel of one
column without noise, which is x-uniform and relaxes to the discrete
hydrostatic state.  Each rising T has its companion; the falling run has one
that follows its stages.  Currents are the collector column of the batch
history, per column of the channel, averaged over the last `avg_t0` ionic
times (t0 = H^2 / K) of each stage.
"""

import json
import time


from . import autotune
from .lbm_ec import HIST_CURRENT, Batch, batch_workspace_bytes, make_params

UNHEALTHY = 5  # history column: nodes with non-finite moments or rho <= 0


def ionic_steps(ny, T, tau_plus=0.8, M=10.0):
    """Steps per ionic time t0 = H^2 / K, K = nu T / M^2 (lattice units)."""
    K = (tau_plus - 0.5) / 3.0 * T / (M * M)
    return ny * ny / K


def stages(T_fall, ny, start_t0, dwell_t0, tau_plus=0.8, M=10.0):
    """The falling run's stages [(T, steps)]: the first T for start_t0 ionic
    times (growth of the vortices), each later T for dwell_t0."""
    out = []
    for k, T in enumerate(T_fall):
        n = (start_t0 if k == 0 else dwell_t0) * ionic_steps(ny, T, tau_plus, M)
        out.append((float(T), int(round(n))))
    return out


def window_mean(history, col, lo, hi):
    """Mean of history[:, col] over the rows with lo < step <= hi."""
    rows = history[(history[:, 0] > lo) & (history[:, 0] <= hi)]
    if len(rows) == 0:
        return float("nan")
    return float(rows[:, col].mean())


def ne0(hist_run, nx_run, hist_comp, nx_comp, lo, hi):
    """Ne_0 over the window (lo, hi]: collector current per column of the run
    over that of its hydrostatic companion."""
    i = window_mean(hist_run, HIST_CURRENT, lo, hi) / nx_run
    i0 = window_mean(hist_comp, HIST_CURRENT, lo, hi) / nx_comp
    return i / i0


def bracket_rising(Ts, ne, thr):
    """(T_below, T_above) around the onset: the highest T still hydrostatic
    below the lowest T with Ne_0 > 1 + thr (None where it does not exist)."""
    pairs = sorted(zip(Ts, ne))
    above = [T for T, v in pairs if v > 1.0 + thr]
    if not above:
        return (max(Ts), None)
    t_hi = min(above)
    below = [T for T, v in pairs if T < t_hi]
    return (max(below) if below else None, t_hi)


def bracket_falling(Ts, ne, thr):
    """(T_below, T_above) around the return to the hydrostatic state along the
    falling stages: the first stage with Ne_0 <= 1 + thr and the stage before
    it (None where the run never returns or never convected)."""
    for k, (T, v) in enumerate(zip(Ts, ne)):
        if v <= 1.0 + thr:
            return (T, Ts[k - 1] if k > 0 else None)
    return (None, Ts[-1] if Ts else None)


def run(nx=61, ny=50, T_rise=(100, 110, 120, 130, 140, 150, 155, 160, 165, 170, 180, 200),
        T_fall=(200, 190, 180, 170, 160, 150, 140, 130, 120, 115, 110, 105, 100), start_t0=12.0, dwell_t0=4.0,
        avg_t0=1.0, thr=0.01, precision="fp32_f64math", C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8, Lambda=0.25,
        Lambda_g=1e-6, max_rows=4000, device="cuda:0", tuning=None, progress=None):
    common = dict(C=C, M=M, Fe=Fe, tau_plus=tau_plus, Lambda=Lambda, Lambda_g=Lambda_g, precision=precision)
    plan = stages(T_fall, ny, start_t0, dwell_t0, tau_plus, M)
    total = sum(n for _, n in plan)
    emit = max(1, total // max_rows)
    hist_rows = total // emit + 2
    cfgs = []
    for i, T in enumerate(T_rise):
        cfgs.append(("rise", float(T), dict(nx=nx, ny=ny, T=float(T), init_mode="eq29", instance_id=i, **common)))
        cfgs.append(("rise0", float(T), dict(nx=1, ny=ny, T=float(T), init_mode="noise", noise_amp=0.0, **common)))
    T0 = plan[0][0]
    cfgs.append(("fall", T0, dict(nx=nx, ny=ny, T=T0, init_mode="eq29", instance_id=len(T_rise), **common)))
    cfgs.append(("fall0", T0, dict(nx=1, ny=ny, T=T0, init_mode="noise", noise_amp=0.0, **common)))
    if tuning is None:
        # launch shapes for this composition, timed on a throwaway batch
        # before the clock starts (they never change results)
        tuning = autotune.tune_batch([c for _, _, c in cfgs], device=device)
    params = [make_params(**c) for _, _, c in cfgs]
    ws = batch_workspace_bytes(params, len(cfgs), hist_rows) + (1 << 20)
    b = Batch(len(cfgs), ws, precision=precision, emit_every=emit, hist_rows=hist_rows, device=device)
    b.set_tuning(*tuning)
    slots = [b.admit(total, **c) for _, _, c in cfgs]
    if None in slots:
        raise RuntimeError("batch workspace too small")
    kind = {k: s for (k, _, _), s in zip(cfgs, slots) if k in ("fall", "fall0")}
    b.stream.synchronize()
    t = time.perf_counter()
    ends, done = [], 0
    for k, (T, n) in enumerate(plan):
        if k > 0:
            b.set_T(kind["fall"], T)
            b.set_T(kind["fall0"], T)
        b.step(n)
        done += n
        ends.append(done)
        if progress is not None:
            b.stream.synchronize()
            progress(f"stage T = {T:g}: {n} steps, {done} of {total}, {time.perf_counter() - t:.1f} s")
    b.stream.synchronize()
    seconds = time.perf_counter() - t
    assert sorted(b.poll()) == sorted(slots)
    hist = {s: b.history(s) for s in slots}
    nodes = sum(c["nx"] * c["ny"] for _, _, c in cfgs)
    b.close()

    healthy = all(h[:, UNHEALTHY].max() == 0 for h in hist.values())
    rise, comp = {}, {}
    for (k, T, c), s in zip(cfgs, slots):
        if k == "rise":
            rise[T] = s
        elif k == "rise0":
            comp[T] = s
    avg = lambda T: avg_t0 * ionic_steps(ny, T, tau_plus, M)
    ne_rise = [ne0(hist[rise[T]], nx, hist[comp[T]], 1, total - avg(T), total) for T in sorted(rise)]
    Ts_fall = [T for T, _ in plan]
    ne_fall = [ne0(hist[kind["fall"]], nx, hist[kind["fall0"]], 1, e - avg(T), e) for (T, _), e in zip(plan, ends)]
    return dict(
        grid=[nx, ny], precision=precision, steps=total, emit_every=emit, slots=len(cfgs), seconds=seconds,
        us_per_step=seconds / total * 1e6, mlups=nodes * total / seconds / 1e6, healthy=healthy,
        rising=[[T, v] for T, v in zip(sorted(rise), ne_rise)],
        falling=[[T, v] for T, v in zip(Ts_fall, ne_fall)],
        T_c_bracket=list(bracket_rising(sorted(rise), ne_rise, thr)),
        T_f_bracket=list(bracket_falling(Ts_fall, ne_fall, thr)),
        threshold=thr, start_t0=start_t0, dwell_t0=dwell_t0, avg_t0=avg_t0, tuning=list(tuning),
    )


def main(argv=None):
    """Command line: runs both branches as one batch and prints one JSON line
    (Ne_0 per T on each branch, the brackets of T_c and T_f, the run time)."""
    import argparse

    floats = lambda s: [float(v) for v in s.split(",")]
    ap = argparse.ArgumentParser(description="Ne_0(T) hysteresis: rising and falling branches in one batch")
    ap.add_argument("--nx", type=int, default=61)
    ap.add_argument("--ny", type=int, default=50)
    ap.add_argument("--rise", type=floats, default=None, help="T values of the rising branch (comma separated)")
    ap.add_argument("--fall", type=floats, default=None, help="T stages of the falling branch, first the highest")
    ap.add_argument("--start-t0", type=float, default=12.0, help="ionic times at the first falling stage")
    ap.add_argument("--dwell-t0", type=float, default=4.0, help="ionic times at each later stage")
    ap.add_argument("--precision", default="fp32_f64math", choices=["fp64", "fp32", "fp32_f64math"])
    ap.add_argument("--tuning", default=None, help="fft_threads,collide_bx,collide_by[,collide_tw] (default: autotuned)")
    ap.add_argument("--Lambda", type=float, default=0.25, help="fluid TRT parameter of Eq. 17 (the paper's is 1/12)")
    ap.add_argument("--tau-plus", type=float, default=0.8, help="fluid tau+")
    args = ap.parse_args(argv)
    kw = {"Lambda": args.Lambda, "tau_plus": args.tau_plus}
    if args.rise:
        kw["T_rise"] = args.rise
    if args.fall:
        kw["T_fall"] = args.fall
    if args.tuning:
        kw["tuning"] = tuple(int(v) for v in args.tuning.split(","))
    import sys

    res = run(nx=args.nx, ny=args.ny, start_t0=args.start_t0, dwell_t0=args.dwell_t0, precision=args.precision,
              progress=lambda m: print(m, file=sys.stderr, flush=True), **kw)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
