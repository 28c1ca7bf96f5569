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
    MALLOC_MMAP_MAX_=0 MALLOC_TRIM_THRESHOLD_=68719476736 \
        python tests/golden/make_oracle_golden.py cfg2 --threads 7

With --threads the collision of each step (86 % of an oracle step at these
sizes: pointwise, node by node) is handed to the oracle's own Oracle.collide
in bands of rows on a thread pool, and the oracle's node-wise moments, row
transforms and per-wavenumber Thomas solve run on bands of rows (or
wavenumber columns) as well; the rest (mean mode, field, streaming) is the
oracle's call on the whole grid.  Each of these computes an element from its
own node, row or column alone, so the bands give the same floating-point
operations on the same operands as one call on the grid:
tests/test_golden_slab_driver.py checks the two bit for bit.  The glibc
settings keep freed arrays in the heap for the next step (fresh GB-sized
arrays otherwise cost about half of each step in page faults at this size);
they change no arithmetic.
"""

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Oracle, Params, lbm, poisson  # noqa: E402

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
BAND_ROWS = 4


class _Band:
    """The state Oracle.collide reads (lattice constants, f, g), restricted
    to rows [a, b) as views of the oracle's own arrays."""

    def __init__(self, o, a, b):
        self.lc = o.lc
        self.ft = o.ft[:, a:b]
        self.gt = o.gt[:, a:b]


def _row_banded(fn, pool, bands, lead):
    """fn applied band by band along the row axis (axis `lead` of its array
    arguments; `lead` = 1 for population stacks (9, ny, nx), 0 for fields
    (ny, nx)), the results written into one output per return value."""

    def wrapped(*args):
        def part(ab):
            a, b = ab
            return fn(*[x[:, a:b] if (lead == 1 and x.ndim == 3) else x[a:b] for x in args])

        parts = list(pool.map(part, bands))
        first = parts[0]
        if isinstance(first, tuple):
            return tuple(np.concatenate([p[i] for p in parts], axis=0) for i in range(len(first)))
        return np.concatenate(parts, axis=0)

    return wrapped


def _column_banded(fn, pool, ncols, width=256):
    """fn of (n, nx) arrays, independent per trailing index, applied to
    bands of columns."""
    bands = [(a, min(a + width, ncols)) for a in range(0, ncols, width)]

    def wrapped(*args):
        parts = list(pool.map(lambda ab: fn(*[x[:, ab[0]:ab[1]] for x in args]), bands))
        return np.concatenate(parts, axis=1)

    return wrapped


class _BandedMoments:
    """Within the block, the oracle's node-wise moments (Eq. 5-7), its row
    transforms (Eq. 19) and its per-wavenumber Thomas solve run band by band
    on the pool: the module functions Oracle.macroscopic reaches are swapped
    for wrappers that call the originals on bands of rows (or, for the
    Thomas solve, of wavenumber columns) and stack the results; every
    element is computed by the same function from the same operands."""

    def __init__(self, o, pool, bands):
        nx = o.p.nx
        self.swaps = [
            (lbm, "charge_deviation", _row_banded(lbm.charge_deviation, pool, bands, 1)),
            (lbm, "density_deviation", _row_banded(lbm.density_deviation, pool, bands, 1)),
            (lbm, "velocity", _row_banded(lbm.velocity, pool, bands, 1)),
            (poisson, "dft_x", _row_banded(poisson.dft_x, pool, bands, 0)),
            (poisson, "idft_x", _row_banded(poisson.idft_x, pool, bands, 0)),
            (poisson, "thomas", _column_banded(poisson.thomas, pool, nx)),
        ]
        self.saved = []

    def __enter__(self):
        for mod, name, fn in self.swaps:
            self.saved.append((mod, name, getattr(mod, name)))
            setattr(mod, name, fn)
        return self

    def __exit__(self, *exc):
        for mod, name, fn in self.saved:
            setattr(mod, name, fn)
        return False


def step_in_bands(o, pool, n=1, band_rows=BAND_ROWS):
    """n steps of o, each Oracle.step's sequence (moments, collision,
    streaming) with the collision called band by band on the pool, and the
    moments' node-wise parts and row transforms in bands as well."""
    if o.pending_T is not None:
        raise ValueError("a pending change of T is left to Oracle.step")
    ny = o.p.ny
    bands = [(a, min(a + band_rows, ny)) for a in range(0, ny, band_rows)]
    mbands = [(a, min(a + 4 * band_rows, ny)) for a in range(0, ny, 4 * band_rows)]
    for _ in range(n):
        with _BandedMoments(o, pool, mbands):
            m = o.macroscopic()
        ft_post = np.empty_like(o.ft)
        gt_post = np.empty_like(o.gt)

        def collide_band(ab):
            a, b = ab
            mb = {k: (v[a:b] if np.ndim(v) == 2 else v) for k, v in m.items()}
            ft_post[:, a:b], gt_post[:, a:b] = Oracle.collide(_Band(o, a, b), mb)

        list(pool.map(collide_band, bands))
        del m
        fs = pool.submit(lbm.stream_fluid, ft_post, o.s_ref)
        gs = pool.submit(lbm.stream_charge, gt_post, o.R, o.lc.rho0)
        o.ft, o.gt = fs.result(), gs.result()
        o.n += 1
    return o


def sample_rows(ny, stride):
    """Every stride-th row, plus the rows next to both electrodes."""
    rows = sorted(set(list(range(0, ny, stride)) + [1, ny - 2, ny - 1]))
    return np.array(rows)


def sample_cols(nx, stride):
    """Every stride-th column, plus column 1 and the periodic-wrap column nx-1."""
    cols = sorted(set(list(range(0, nx, stride)) + [1, nx - 1]))
    return np.array(cols)


def main(name, threads=0):
    case = CASES[name]
    p = Params(**case["params"])
    o = Oracle(p)
    pool = ThreadPoolExecutor(threads) if threads > 1 else None
    rows = sample_rows(p.ny, case["stride"])
    cols = sample_cols(p.nx, case["stride"])
    out = {"rows": rows, "cols": cols}
    path = os.path.join(HERE, f"oracle_{name}.npz")
    meta = dict(case=name, params=case["params"], snapshots=[], stride=case["stride"],
                generator="tests/golden/make_oracle_golden.py (oracle only)")
    t = time.time()
    for snap in case["snapshots"]:
        while o.n < snap:
            k = min(50, snap - o.n)
            if pool is None:
                o.step(k)
            else:
                step_in_bands(o, pool, k)
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
    ap = argparse.ArgumentParser()
    ap.add_argument("case", choices=sorted(CASES))
    ap.add_argument("--threads", type=int, default=0,
                    help="collide in bands of rows on this many threads (0: Oracle.step)")
    a = ap.parse_args()
    main(a.case, a.threads)
