"""Writes oracle reference fields for the large parity cases.

Calls only the oracle (oracle/), never the HIP path.  For each named case the
oracle runs the full grid for the stated number of steps and the script
stores, for each snapshot step, the fields on a regular subsample (every
`stride`-th row and column, plus the first and last rows), together with
max |X| over the full grid so that relative errors normalise exactly as the
full comparison would.

    python tests/golden/make_oracle_golden.py cfg1      # 1024 x 840, 10000 steps
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
    # bandwidth configuration 4096 x 4096, T = 500, noise 1e-4; a 100-step prefix
    "cfg2_prefix": dict(params=dict(nx=4096, ny=4096, T=500.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8,
                                    Lambda=0.25, Lambda_g=1e-6, noise_amp=1e-4, seed=181205711),
                        snapshots=[100], stride=16),
}


def sample_rows(ny, stride):
    rows = sorted(set(list(range(0, ny, stride)) + [ny - 1]))
    return np.array(rows)


def main(name):
    case = CASES[name]
    p = Params(**case["params"])
    o = Oracle(p)
    rows = sample_rows(p.ny, case["stride"])
    cols = np.arange(0, p.nx, case["stride"])
    out = {"rows": rows, "cols": cols}
    t = time.time()
    for snap in case["snapshots"]:
        o.step(snap - o.n)
        f = o.fields()
        for k in ("rho", "ux", "uy", "rho_c", "phi"):
            out[f"{k}_{snap}"] = f[k][np.ix_(rows, cols)]
            out[f"max_{k}_{snap}"] = np.max(np.abs(f[k]))
        out[f"max_u_{snap}"] = np.max(np.hypot(f["ux"], f["uy"]))
        print(f"{name}: step {snap} done after {time.time() - t:.0f} s", flush=True)
    path = os.path.join(HERE, f"oracle_{name}.npz")
    np.savez_compressed(path, **out)
    meta = dict(case=name, params=case["params"], snapshots=case["snapshots"], stride=case["stride"],
                generator="tests/golden/make_oracle_golden.py (oracle only)")
    with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as fh:
        json.dump(meta, fh, indent=1)
    print(f"wrote {path}")


if __name__ == "__main__":
    main(sys.argv[1])
