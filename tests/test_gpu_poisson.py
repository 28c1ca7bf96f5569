"""Parity of the Poisson chain alone (x transforms, per-wavenumber y solves
on both interface-solve paths, the x-mean mode) with the oracle's solve,
through lbm_ec_poisson, on seeded charge fields, up to the widest grid
(nx = 8192, the longest x transform one workgroup's LDS holds; a longer
row is refused), with rows that take the first transform pass in registers
(nx = 8 or 16 times the transform threads) and rows that do not.

The y systems split into chunks of 32 rows; the cases give interface
systems of 0 (one chunk), 1, 26, 127 and 256 interfaces (recursive
doubling, 256 is its largest size) and 257 and 514 (serial block
elimination).
Tolerances: FP64 1e-11 relative to max |phi|; FP32 storage 1e-6 (the
m >= 1 modes in FP32 arithmetic, the mean mode in FP64).
"""

import numpy as np
import pytest

from oracle import Params
from oracle.lattice import lattice_constants
from oracle.poisson import solve

pytestmark = pytest.mark.gpu

BASE = dict(T=200.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8, Lambda=0.25, Lambda_g=1e-6, noise_amp=1e-3,
            seed=181205711)
# (61, 50), (122, 30), (77, 40): direct DFT passes of prime radix (61; 7 and 11)
# with the twiddle table copied to LDS; (4094, 24) = 2 x 23 x 89: the copy
# fits beside the FP32 ping-pong buffers, not beside the FP64 ones (there the
# direct passes read the table from global memory)
CASES = [(16, 20), (24, 40), (40, 840), (8, 4096), (6, 8224), (6, 8256), (6, 16480), (2048, 24), (4096, 24),
         (8192, 8), (1000, 24), (122, 30), (61, 50), (77, 40), (4094, 24)]
TOL = {"fp64": 1e-11, "fp32_f64math": 1e-6, "fp32": 1e-6}


def _charge(nx, ny, seed):
    rng = np.random.default_rng(seed)
    y = (np.arange(ny) + 0.5) / ny
    return (np.exp(-3.0 * y)[:, None] * (1.0 + 0.3 * rng.standard_normal((ny, nx)))).astype(np.float64)


@pytest.mark.parametrize("precision", ["fp64", "fp32_f64math", "fp32"])
@pytest.mark.parametrize("nx,ny", CASES)
def test_poisson_matches_oracle(nx, ny, precision):
    import torch

    from paper_1812_05711_amd.lbm_ec import Simulation

    kw = dict(BASE, nx=nx, ny=ny)
    rho_nd = _charge(nx, ny, 7 + nx + ny)
    eps = lattice_constants(Params(**kw)).eps
    phi_o = solve(rho_nd * eps / float(ny) ** 2, eps)
    sim = Simulation(device="cuda:0", precision=precision, **kw)
    phi_g = sim.poisson(torch.from_numpy(rho_nd)).cpu().numpy()
    sim.close()
    err = np.abs(phi_g - phi_o).max() / np.abs(phi_o).max()
    print(nx, ny, precision, f"{err:.2e}", flush=True)
    assert err <= TOL[precision], err


@pytest.mark.parametrize("precision,nx", [("fp64", 8200), ("fp32", 8200), ("fp64", 5122)])
def test_rows_beyond_the_transform_limit_are_refused(precision, nx):
    """Past 8192 points, or an FP64 row with a prime factor above 5 beyond
    5120 points (ping-pong transform), the row pair's transform does not fit
    one workgroup's LDS: EINVAL before anything is allocated."""
    from paper_1812_05711_amd.lbm_ec import EINVAL, LbmEcError, Simulation

    with pytest.raises(LbmEcError) as ei:
        Simulation(device="cuda:0", precision=precision, **dict(BASE, nx=nx, ny=8))
    assert ei.value.code == EINVAL


@pytest.mark.parametrize("threads", [64, 128, 256, 512])
def test_transform_threads_do_not_change_the_potential(threads):
    """The row sums of the x-mean mode and the transforms give the same bits
    for every transform block size (nx = 1024: the first pass in registers
    at 128 threads, through LDS otherwise)."""
    import torch

    from paper_1812_05711_amd.lbm_ec import Simulation

    kw = dict(BASE, nx=1024, ny=40)
    rho_nd = torch.from_numpy(_charge(1024, 40, 11))
    out = []
    for t in (threads, 128):
        sim = Simulation(device="cuda:0", precision="fp64", **kw)
        sim.set_tuning(t, 1024, 1)
        out.append(sim.poisson(rho_nd).cpu().numpy())
        sim.close()
    assert np.array_equal(out[0], out[1])
