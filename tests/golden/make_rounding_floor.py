"""Rounding floor of FP32 population storage: the oracle with its stored
populations (deviations from its reference rows) rounded to FP32 after every
step, against the FP64 oracle.  The largest difference of the velocity
columns of the history rows (rms u_y, max |u|, first x mode of u_y)
relative to the run's largest |u| is what FP32 storage alone costs, whatever
the arithmetic; the GPU's FP32-storage rows are held to a small multiple of
it where it exceeds the 1e-5 gate.

Cases: the batched T sweep's three smallest instances (ids 37, 59, 62; see
make_sweep_golden.py; against their stored FP64 oracle histories, 20000
steps), and the threshold problem of tests/test_gpu_sweep.py ("thr140",
"thr190": 31 x 25, Eq. 29 perturbation, 5400 steps; against an FP64 oracle
run beside it).

Calls only the oracle and the seeded inputs (no HIP path).

    python tests/golden/make_rounding_floor.py 62        # one case per call
    python tests/golden/make_rounding_floor.py thr190
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Oracle, Params  # noqa: E402
from paper_1812_05711_amd.workloads import sweep_configs  # noqa: E402

STEPS, EVERY = 20000, 100
THRESHOLD = dict(nx=31, ny=25, C=10.0, M=10.0, Fe=4000.0, tau_plus=1.0, Lambda=1 / 12, Lambda_g=1e-6,
                 init_mode="eq29", seed=181205711)
THR_STEPS, THR_EVERY = 5400, 50


def fp32(a):
    return a.astype(np.float32).astype(np.float64)


def _row(o):
    f = o.fields()
    ux, uy = f["ux"] * o.lc.u0, f["uy"] * o.lc.u0
    a1 = np.max(np.abs(np.fft.fft(uy, axis=1)[:, 1])) / uy.shape[1]
    return (o.n, np.sqrt(np.mean(uy ** 2)), np.max(np.hypot(ux, uy)), a1)


def threshold_floor(T):
    """Rows of the FP32-storage oracle and of the FP64 oracle, side by side."""
    o = Oracle(Params(T=T, **THRESHOLD))
    r = Oracle(Params(T=T, **THRESHOLD))
    o.ft, o.gt = fp32(o.ft), fp32(o.gt)
    rows, ref = [], []
    while o.n < THR_STEPS:
        for _ in range(THR_EVERY):
            o.step(1)
            o.ft, o.gt = fp32(o.ft), fp32(o.gt)
        r.step(THR_EVERY)
        rows.append(_row(o))
        ref.append(_row(r))
    return np.array(rows), np.array(ref)


def main(case):
    if case.startswith("thr"):
        rows, ref = threshold_floor(float(case[3:]))
        e = np.max(np.abs(rows[:, 1:4] - ref[:, 1:4]), axis=1) / np.max(ref[:, 2])
        _store(case, e)
        return
    i = int(case)
    cfg = sweep_configs()[i]
    o = Oracle(Params(**{k: v for k, v in cfg.items() if k != "precision"}))
    o.ft, o.gt = fp32(o.ft), fp32(o.gt)
    rows = []
    while o.n < STEPS:
        for _ in range(EVERY):
            o.step(1)
            o.ft, o.gt = fp32(o.ft), fp32(o.gt)
        f = o.fields()
        ux, uy = f["ux"] * o.lc.u0, f["uy"] * o.lc.u0
        a1 = np.max(np.abs(np.fft.fft(uy, axis=1)[:, 1])) / uy.shape[1]
        rows.append((o.n, np.sqrt(np.mean(uy ** 2)), np.max(np.hypot(ux, uy)), a1))
    rows = np.array(rows)
    ref = np.load(os.path.join(HERE, f"oracle_sweep_{i}.npz"))["history"]
    e = np.max(np.abs(rows[:, 1:4] - ref[:, [1, 2, 4]]), axis=1) / np.max(ref[:, 2])
    _store(str(i), e)


def _store(key, e):
    path = os.path.join(HERE, "rounding_floor_sweep.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    data[key] = dict(max_velocity_error=float(e.max()), final_velocity_error=float(e[-1]),
                     generator="tests/golden/make_rounding_floor.py (oracle only)")
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    print(key, data[key], flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
