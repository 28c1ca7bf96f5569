"""Writes oracle histories of three instances of the batched T sweep (the
smallest ones: instance ids 37, 59, 62 of the seeded list, ny 65, 66, 72) for
the parity test of the sweep batch.

Calls only the oracle (oracle/) and the seeded instance list
(paper_1812_05711_amd/workloads.py, which holds no arithmetic of the method),
never the HIP path.  Every 100 steps of the 20000, the quantities the batch
records, in lattice units: step, rms u_y, max |u|, sum of rho_c, the amplitude
of the first x mode of u_y (largest over the rows), 0, the collector current.

    python tests/golden/make_sweep_golden.py 37     # one instance per call
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Oracle, Params  # noqa: E402
from paper_1812_05711_amd.workloads import sweep_configs  # noqa: E402

IDS = (37, 59, 62)
STEPS, EVERY = 20000, 100


def main(i):
    cfg = sweep_configs()[i]
    kw = {k: v for k, v in cfg.items() if k != "precision"}
    o = Oracle(Params(**kw))
    rows = []
    t = time.time()
    while o.n < STEPS:
        o.step(EVERY)
        f = o.fields()
        u0 = o.lc.u0
        ux, uy = f["ux"] * u0, f["uy"] * u0
        rho_c = f["rho_c"] * o.lc.eps / o.lc.H ** 2
        a1 = np.max(np.abs(np.fft.fft(uy, axis=1)[:, 1])) / uy.shape[1]
        _, collector = o.electrode_currents()
        rows.append((o.n, np.sqrt(np.mean(uy ** 2)), np.max(np.hypot(ux, uy)), np.sum(rho_c), a1, 0.0, collector))
        if o.n % 2000 == 0:
            print(f"instance {i}: step {o.n} after {time.time() - t:.0f} s", flush=True)
    path = os.path.join(HERE, f"oracle_sweep_{i}.npz")
    np.savez_compressed(path, history=np.array(rows), t0=o.lc.t0)
    with open(os.path.join(HERE, f"oracle_sweep_{i}.json"), "w") as fh:
        json.dump(dict(instance=i, params=kw, steps=STEPS, emit_every=EVERY,
                       generator="tests/golden/make_sweep_golden.py (oracle only)"), fh, indent=1)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]))
