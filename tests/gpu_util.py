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
    """Relative max errors per field, the velocity as a vector field too.

    rho_m1 = rho - 1 (when both sides give it) is normalised by its own
    max |rho - 1| (1e-5 .. 1e-3), so the hydrostatic density departure is
    gated at the same relative tolerance as the other fields; rho itself is
    normalised by max |rho| ~ 1."""
    e = {k: rel_max_error(g[k], o[k]) for k in FIELDS}
    if "rho_m1" in g and "rho_m1" in o:
        e["rho_m1"] = rel_max_error(g["rho_m1"], o["rho_m1"])
    du = np.hypot(g["ux"] - o["ux"], g["uy"] - o["uy"]).max()
    e["u"] = float(du / max(np.hypot(o["ux"], o["uy"]).max(), 1e-300))
    return e
