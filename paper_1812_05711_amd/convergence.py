"""Grid convergence of the hydrostatic state (section IV.4 states 2nd-order
accuracy in space; section V.1, Fig. 1 and Table II, compare C = 0.1 and
C = 10 with the closed form of Eq. 27-28).

x-uniform channels (one column, no noise) at several ny, all slots of one
batch, run for `n_t0` ionic times (t0 = ny^2 / K) to their steady state.  The
steady state depends on C and Fe only; T = 1200 and tau+ = 1 (K = 2) keep the
ionic time at ny^2 / 2 steps.  Profiles are nondimensional, at the nodes
y_j = (j + 1/2) / ny: rho_c from the fields, E_y = -d phi / dy by the central
differences of the collision with its ghost rows (phi(-1) = 2 - phi(0),
phi(ny) = -phi(ny - 1)).

Self-convergence: each profile against the next finer one restricted to the
coarse nodes (the mean of the two fine nodes around each coarse node, itself
2nd-order accurate), relative L2; the observed order is log2 of the ratio of
successive differences.
"""

import json
import math
import time

import numpy as np

from .lbm_ec import Batch, batch_workspace_bytes, make_params

PARAMS = dict(T=1200.0, M=10.0, Fe=4000.0, tau_plus=1.0, Lambda=0.25, Lambda_g=1e-6)


def ionic_steps(ny, T=PARAMS["T"], tau_plus=PARAMS["tau_plus"], M=PARAMS["M"]):
    K = (tau_plus - 0.5) / 3.0 * T / (M * M)
    return ny * ny / K


def field_from_potential(phi):
    """E_y at the nodes from the nondimensional potential of one column."""
    ny = len(phi)
    ext = np.concatenate([[2.0 - phi[0]], phi, [-phi[-1]]])
    return -(ext[2:] - ext[:-2]) * ny / 2.0


def restrict(fine):
    """Fine-grid nodal values (2n) at the coarse nodes (n): pair means."""
    return 0.5 * (fine[0::2] + fine[1::2])


def rel_l2(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b**2)))


def self_convergence(profiles):
    """profiles: {ny: array} for ny doubling.  Returns [(ny, e, order)]: e the
    relative L2 difference to the next finer grid, order log2(e / e_next)."""
    nys = sorted(profiles)
    e = []
    for a, b in zip(nys[:-1], nys[1:]):
        if b != 2 * a:
            raise ValueError("grids must double")
        e.append((a, rel_l2(profiles[a], restrict(profiles[b]))))
    out = []
    for k, (ny, v) in enumerate(e):
        order = math.log2(v / e[k + 1][1]) if k + 1 < len(e) else None
        out.append((ny, v, order))
    return out


def run(nys=(50, 100, 200, 400, 800), Cs=(0.1, 10.0), n_t0=4.0, precision="fp64", device="cuda:0"):
    """Steady profiles {C: {ny: (E_y, rho_c)}} and the run time."""
    cfgs = [dict(nx=1, ny=int(ny), C=float(C), init_mode="noise", noise_amp=0.0, precision=precision, **PARAMS)
            for C in Cs for ny in nys]
    steps = [int(round(n_t0 * ionic_steps(c["ny"]))) for c in cfgs]
    params = [make_params(**c) for c in cfgs]
    ws = batch_workspace_bytes(params, len(cfgs), 4) + (1 << 20)
    b = Batch(len(cfgs), ws, precision=precision, emit_every=0, hist_rows=4, device=device)
    slots = [b.admit(n, **c) for n, c in zip(steps, cfgs)]
    if None in slots:
        raise RuntimeError("batch workspace too small")
    b.stream.synchronize()
    t = time.perf_counter()
    b.step(max(steps))
    b.stream.synchronize()
    seconds = time.perf_counter() - t
    assert sorted(b.poll()) == sorted(slots)
    out = {}
    for c, s in zip(cfgs, slots):
        f = b.fields(s)
        phi = f["phi"][:, 0].cpu().numpy()
        rc = f["rho_c"][:, 0].cpu().numpy()
        out.setdefault(c["C"], {})[c["ny"]] = (field_from_potential(phi), rc)
    b.close()
    return out, dict(seconds=seconds, steps=max(steps), slots=len(cfgs), n_t0=n_t0, precision=precision)


def main(argv=None):
    """Command line: one JSON line with the self-convergence of E_y and rho_c
    per C (difference to the next finer grid and the observed order)."""
    import argparse

    ap = argparse.ArgumentParser(description="grid convergence of the hydrostatic state (one batch)")
    ap.add_argument("--ny", default="50,100,200,400,800", help="doubling row counts")
    ap.add_argument("--t0", type=float, default=4.0, help="ionic times per run")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "fp32_f64math"])
    args = ap.parse_args(argv)
    nys = [int(v) for v in args.ny.split(",")]
    prof, info = run(nys=nys, n_t0=args.t0, precision=args.precision)
    res = dict(info)
    for C, byny in prof.items():
        res[f"C={C:g}"] = {
            "E_y": [[ny, e, o] for ny, e, o in self_convergence({n: v[0] for n, v in byny.items()})],
            "rho_c": [[ny, e, o] for ny, e, o in self_convergence({n: v[1] for n, v in byny.items()})],
        }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
