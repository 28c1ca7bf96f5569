"""The paper's spectral y route (Eq. 21-25, lbm_ec_set_y_solver) against the
oracle's solve and against the chunked tridiagonal route, through the C ABI.

Column lengths 2 ny cover register radices only (40, 100, 2048), a generic
prime pass (74 = 2 x 37, 1680 with a factor 7), the largest ny the LDS
admits in each storage type (2560 in FP64, 5120 in FP32; one more row is
refused), and channels with no m >= 1 mode (nx = 1) or only the Nyquist one
(nx = 2).  Tolerances as for the Poisson chain: FP64 1e-11 relative to
max |phi|, FP32 storage 1e-6; coupled steps as in the parity tests.
"""

import numpy as np
import pytest

from gpu_util import errors, oracle_fields
from oracle import Params
from oracle.lattice import lattice_constants
from oracle.poisson import solve

pytestmark = pytest.mark.gpu

BASE = dict(T=200.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8, Lambda=0.25, Lambda_g=1e-6, noise_amp=1e-3,
            seed=181205711)
TOL = {"fp64": 1e-11, "fp32_f64math": 1e-6, "fp32": 1e-6}
CASES = [(16, 20), (24, 37), (122, 20), (61, 50), (1, 16), (2, 9), (40, 840)]


def _charge(nx, ny, seed):
    rng = np.random.default_rng(seed)
    y = (np.arange(ny) + 0.5) / ny
    return (np.exp(-3.0 * y)[:, None] * (1.0 + 0.3 * rng.standard_normal((ny, nx)))).astype(np.float64)


def _poisson(kw, precision, solver, rho_nd):
    import torch

    from paper_1812_05711_amd.lbm_ec import Simulation

    sim = Simulation(device="cuda:0", precision=precision, **kw)
    sim.set_y_solver(solver)
    phi = sim.poisson(torch.from_numpy(rho_nd)).cpu().numpy()
    sim.close()
    return phi


@pytest.mark.parametrize("precision", ["fp64", "fp32_f64math", "fp32"])
@pytest.mark.parametrize("nx,ny", CASES + [(64, 2560), (8, 5120)])
def test_spectral_poisson_matches_oracle(nx, ny, precision):
    if precision == "fp64" and ny > 2560:
        return  # beyond the FP64 limit (refused below)
    kw = dict(BASE, nx=nx, ny=ny)
    print("yspec", nx, ny, precision, flush=True)
    rho_nd = _charge(nx, ny, 11 + nx + ny)
    eps = lattice_constants(Params(**kw)).eps
    phi_o = solve(rho_nd * eps / float(ny) ** 2, eps)
    phi_g = _poisson(kw, precision, "spectral", rho_nd)
    err = np.abs(phi_g - phi_o).max() / np.abs(phi_o).max()
    print(f"  {err:.2e}", flush=True)
    assert err <= TOL[precision], err


@pytest.mark.parametrize("nx,ny", [(24, 37), (61, 50), (40, 840)])
def test_spectral_and_tridiagonal_agree_to_rounding(nx, ny):
    kw = dict(BASE, nx=nx, ny=ny)
    rho_nd = _charge(nx, ny, 3)
    a = _poisson(kw, "fp64", "spectral", rho_nd)
    b = _poisson(kw, "fp64", "tridiagonal", rho_nd)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32_f64math", 1e-5)])
@pytest.mark.parametrize("nx,ny,steps", [(24, 20, 40), (61, 50, 30)])
def test_coupled_steps_with_spectral_y(nx, ny, steps, precision, tol):
    import torch

    from paper_1812_05711_amd.lbm_ec import Simulation

    kw = dict(BASE, nx=nx, ny=ny)
    o = oracle_fields(kw, steps)
    sim = Simulation(device="cuda:0", precision=precision, **kw)
    sim.set_y_solver("spectral")
    sim.step(steps)
    g = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    torch.cuda.synchronize()
    sim.close()
    e = errors(g, o)
    print(nx, ny, precision, {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    for k in ("rho", "u", "rho_c", "phi"):
        assert e[k] <= tol, (k, e)


def test_refused_solver_and_sizes():
    from paper_1812_05711_amd.lbm_ec import EINVAL, LbmEcError, Simulation

    for precision, ny in (("fp64", 2561), ("fp32", 5121)):
        sim = Simulation(device="cuda:0", precision=precision, **dict(BASE, nx=4, ny=ny))
        with pytest.raises(LbmEcError) as ei:
            sim.set_y_solver("spectral")
        assert ei.value.code == EINVAL
        sim.close()
    sim = Simulation(device="cuda:0", precision="fp64", **dict(BASE, nx=4, ny=12))
    with pytest.raises(LbmEcError) as ei:
        sim.set_y_solver(7)
    assert ei.value.code == EINVAL
    sim.close()


def test_spectral_y_with_a_change_of_T():
    """lbm_ec_set_T rewrites the tables of the new T and leaves the spectral
    route's own (T-independent) twiddles in place."""
    import torch

    from oracle import Oracle
    from paper_1812_05711_amd.lbm_ec import Simulation

    kw = dict(BASE, nx=24, ny=20)
    o = Oracle(Params(**kw))
    o.step(15)
    o.set_T(150.0)
    o.step(20)
    sim = Simulation(device="cuda:0", precision="fp64", **kw)
    sim.set_y_solver("spectral")
    sim.step(15)
    sim.set_T(150.0)
    sim.step(20)
    g = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    torch.cuda.synchronize()
    sim.close()
    e = errors(g, o.fields())
    for k in ("rho", "u", "rho_c", "phi"):
        assert e[k] <= 1e-11, (k, e)
