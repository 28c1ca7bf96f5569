"""Writes oracle reference fields for the large parity cases.

Calls only the oracle (oracle/), never the HIP path.  For each named case the
oracle runs the full grid for the stated number of steps and the script
stores, for each snapshot step, the fields on a regular subsample (every
`stride`-th row and column, plus the rows next to both electrodes and the
columns 1 and nx - 1, where the periodic wrap is used), together with
max |X| over the full grid so that relative errors normalise exactly as the
full comparison would.

    python tests/golden/make_oracle_golden.py cfg1      # 1024 x 840, 10000 steps
    python tests/golden/make_oracle_golden.py cfg2      # 4096 x 4096, 1000 steps
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Oracle, Params  # noqa: E402

CASES = {
    # single-instance FP64 vs FP32-deviation configuration: T = 300, C = 10,
    # M = 10, Fe = 4000, noise 1e-3, 10000 steps
    "cfg1": dict(params=dict(nx=1024, ny=840, T=300.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8,
                             Lambda=0.25, Lambda_g=1e-6, noise_amp=1e-3, seed=181205711),
                 snapshots=[1000, 10000], stride=8),
    # bandwidth configuration 4096 x 4096, T = 500, noise 1e-4, 1000 steps,
    # with a snapshot of the 100-step prefix as well
    "cfg2": dict(params=dict(nx=4096, ny=4096, T=500.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8,
                             Lambda=0.25, Lambda_g=1e-6, noise_amp=1e-4, seed=181205711),
                 snapshots=[100, 1000], stride=16),
}

FIELDS = ("rho", "rho_m1", "ux", "uy", "rho_c", "phi")


def sample_rows(ny, stride):
    """Every stride-th row, plus the rows next to both electrodes."""
    rows = sorted(set(list(range(0, ny, stride)) + [1, ny - 2, ny - 1]))
    return np.array(rows)


def sample_cols(nx, stride):
    """Every stride-th column, plus column 1 and the periodic-wrap column nx-1."""
    cols = sorted(set(list(range(0, nx, stride)) + [1, nx - 1]))
    return np.array(cols)


def main(name):
    case = CASES[name]
    p = Params(**case["params"])
    o = Oracle(p)
    rows = sample_rows(p.ny, case["stride"])
    cols = sample_cols(p.nx, case["stride"])
    out = {"rows": rows, "cols": cols}
    path = os.path.join(HERE, f"oracle_{name}.npz")
    meta = dict(case=name, params=case["params"], snapshots=[], stride=case["stride"],
                generator="tests/golden/make_oracle_golden.py (oracle only)")
    t = time.time()
    for snap in case["snapshots"]:
        while o.n < snap:
            o.step(min(50, snap - o.n))
            print(f"{name}: step {o.n} after {time.time() - t:.0f} s", flush=True)
        f = o.fields()
        for k in FIELDS:
            out[f"{k}_{snap}"] = f[k][np.ix_(rows, cols)]
            out[f"max_{k}_{snap}"] = np.max(np.abs(f[k]))
        out[f"max_u_{snap}"] = np.max(np.hypot(f["ux"], f["uy"]))
        del f
        # written after every snapshot, so that a long run keeps what it has
        np.savez_compressed(path, **out)
        meta["snapshots"].append(snap)
        with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as fh:
            json.dump(meta, fh, indent=1)
        print(f"{name}: step {snap} written after {time.time() - t:.0f} s", flush=True)
    print(f"wrote {path}")


if __name__ == "__main__":
    main(sys.argv[1])
