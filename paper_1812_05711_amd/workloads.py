"""Seeded synthetic workloads of the benchmark and the tests: instance lists
and their sizes only (no arithmetic of the method), shared by the GPU path
and the oracle's reference runs.

T sweep: n instances, ny uniform in ny_range (seeded), nx the smallest
5-smooth length not below round(1.22 ny) (the aspect ratio 1.22 of the
paper's domain, section V.2; a periodic box cannot be zero-padded, so the
period is that length), T uniform in T_range, shared C, M, Fe and
precision, the charge noise of the hydrostatic start seeded per instance.
"""

import numpy as np


def five_smooth_at_least(n: int) -> int:
    m = max(1, int(n))
    while True:
        k = m
        for p in (2, 3, 5):
            while k % p == 0:
                k //= p
        if k == 1:
            return m
        m += 1


def sweep_configs(n=64, seed=181205711, ny_range=(64, 256), T_range=(100.0, 250.0), C=10.0, M=10.0, Fe=4000.0,
                  tau_plus=0.8, Lambda=0.25, Lambda_g=1e-6, noise_amp=1e-3, precision="fp32_f64math"):
    """The seeded instance list of a sweep (dicts of simulation parameters)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        ny = int(rng.integers(ny_range[0], ny_range[1] + 1))
        nx = five_smooth_at_least(round(1.22 * ny))
        T = float(rng.uniform(*T_range))
        out.append(dict(nx=nx, ny=ny, T=T, C=C, M=M, Fe=Fe, tau_plus=tau_plus, Lambda=Lambda, Lambda_g=Lambda_g,
                        noise_amp=noise_amp, seed=seed, instance_id=i, precision=precision))
    return out
