"""Rounding floor of FP32 population storage on the batched T sweep's three
smallest instances (ids 37, 59, 62; see make_sweep_golden.py): the oracle
with its stored populations (deviations from its reference rows) rounded to
FP32 after every step, against the FP64 oracle history.  The largest
difference of the velocity columns (rms u_y, max |u|, first x mode of u_y)
relative to the run's largest |u| is what FP32 storage alone costs, whatever
the arithmetic; the GPU's FP32-storage rows are held to a small multiple of
it where it exceeds the 1e-5 gate.

Calls only the oracle and the seeded instance list (no HIP path).

    python tests/golden/make_rounding_floor.py 62     # one instance per call
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


def fp32(a):
    return a.astype(np.float32).astype(np.float64)


def main(i):
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
    path = os.path.join(HERE, "rounding_floor_sweep.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    data[str(i)] = dict(max_velocity_error=float(e.max()), final_velocity_error=float(e[-1]),
                        generator="tests/golden/make_rounding_floor.py (oracle only)")
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    print(i, data[str(i)], flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]))
