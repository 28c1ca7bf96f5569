"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and the oracle on the same seeded parameters, and compare fields."""

import numpy as np

from oracle import Oracle, Params
from oracle.diagnostics import rel_max_error

FIELDS = ("rho", "ux", "uy", "rho_c", "phi")


def oracle_fields(kw, steps):
    p = Params(**{k: v for k, v in kw.items() if k != "precision"})
    o = Oracle(p)
    o.step(steps)
    return o.fields()


def gpu_fields(kw, steps, chunks=1):
    from paper_1812_05711_amd.lbm_ec import Simulation
    import torch

    sim = Simulation(device="cuda:0", **kw)
    left = steps
    per = max(1, steps // chunks) if steps else 0
    while left > 0:
        n = min(per, left)
        sim.step(n)
        left -= n
    f = sim.fields()
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in f.items()}
    out["steps"] = sim.steps_done()
    sim.close()
    return out


def errors(g, o):
    """Relative max errors per field, the velocity as a vector field too."""
    e = {k: rel_max_error(g[k], o[k]) for k in FIELDS}
    du = np.hypot(g["ux"] - o["ux"], g["uy"] - o["uy"]).max()
    e["u"] = float(du / max(np.hypot(o["ux"], o["uy"]).max(), 1e-300))
    return e
