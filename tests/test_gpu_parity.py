"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: FP64 storage 1e-11 relative (max |x - x_oracle| / max |x_oracle|)
on rho, rho - 1 (normalised by its own max), u (as a vector field), rho_c
and phi; FP32-deviation storage 1e-5.
Cases span several wavefronts in x, ragged tails (odd nx, nx not a multiple
of 64), the generic-radix transform (nx = 122 = 2 * 61), the minimal ny = 3,
an x-uniform channel (nx = 1), all three initial states, and the full
122 x 100 configuration over 2000 steps.
"""

import numpy as np
import pytest

from gpu_util import errors, gpu_fields, oracle_fields

pytestmark = pytest.mark.gpu

BASE = dict(T=200.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8, Lambda=0.25, Lambda_g=1e-6,
            noise_amp=1e-3, seed=181205711)
TOL64 = 1e-11
TOL32 = 1e-5


def _check(kw, steps, tol, fields=("rho", "rho_m1", "u", "rho_c", "phi")):
    o = oracle_fields(kw, steps)
    g = gpu_fields(kw, steps)
    assert g["steps"] == steps
    e = errors(g, o)
    print(kw.get("nx"), kw.get("ny"), kw.get("precision", "fp64"), steps, {k: f"{v:.2e}" for k, v in e.items()},
          flush=True)
    for k in fields:
        assert e[k] <= tol, (k, e)
    return e


@pytest.mark.parametrize("nx,ny,steps", [
    (16, 12, 50),
    (15, 10, 30),
    (122, 20, 40),
    (100, 7, 25),
    (8, 3, 10),
    (1, 16, 40),
    (200, 33, 20),
    # collide tiles of 2, 4, 15 and 8 rows, full and partial last tiles
    (8, 520, 30),
    (6, 1100, 20),
    (5, 1027, 20),
    (4, 4000, 10),
    (3, 4200, 10),
    (3, 4100, 10),
])
def test_fp64_small(nx, ny, steps):
    _check(dict(BASE, nx=nx, ny=ny), steps, TOL64)


def test_fp64_step0_is_initial_state():
    _check(dict(BASE, nx=24, ny=10), 0, TOL64)


def test_fp64_eq29_init():
    _check(dict(BASE, nx=48, ny=20, init_mode="eq29", T=170.0, tau_plus=1.0, Lambda=1 / 12), 60, TOL64)


def test_fp64_rest_poiseuille_force():
    kw = dict(BASE, nx=4, ny=8, init_mode="rest", C=0.0, body_force_x=1e-6, tau_plus=1.0, Lambda=3 / 16)
    o = oracle_fields(kw, 200)
    g = gpu_fields(kw, 200)
    e = errors(g, o)
    assert e["ux"] <= TOL64 and e["rho"] <= TOL64, e


def test_fp64_symmetric_rate_reading():
    _check(dict(BASE, nx=20, ny=12, charge_rates="symmetric"), 40, TOL64)


def test_fp64_full_122x100_2000_steps():
    _check(dict(BASE, nx=122, ny=100), 2000, TOL64)


@pytest.mark.parametrize("precision", ["fp32_f64math", "fp32"])
@pytest.mark.parametrize("nx,ny,steps", [(16, 12, 50), (122, 100, 200), (61, 40, 300), (7, 1027, 40)])
def test_fp32_storage_small(nx, ny, steps, precision):
    _check(dict(BASE, nx=nx, ny=ny, precision=precision), steps, TOL32)


@pytest.mark.parametrize("precision,nx", [("fp64", 4096), ("fp64", 8192), ("fp32_f64math", 8192), ("fp32", 8192),
                                          ("fp64", 3000), ("fp32_f64math", 1500)])
def test_widest_grid(precision, nx):
    """Rows wider than one collide tile (1024 columns, halo columns
    recomputed), up to the longest x transform a workgroup's LDS holds
    (8192 points in either storage type), and ragged last tiles (3000 =
    2 x 1024 + 952, 1500 = 1024 + 476)."""
    _check(dict(BASE, nx=nx, ny=12, precision=precision), 20, TOL64 if precision == "fp64" else TOL32)


def test_widest_grid_fp64_tall():
    """The 4096-wide row in FP64 over several tile bands (ny = 520: two-row
    bands), so that tile edges in x and y meet."""
    _check(dict(BASE, nx=4096, ny=520), 6, TOL64)


def test_fp32_f64math_full_122x100_2000_steps():
    _check(dict(BASE, nx=122, ny=100, precision="fp32_f64math"), 2000, TOL32)


def test_mass_conserved_on_device():
    """sum(rho - 1) over the channel stays constant (bounce-back walls and a
    source with zero mass), read through the FP64 device reduction."""
    from paper_1812_05711_amd.lbm_ec import Simulation

    sim = Simulation(device="cuda:0", **dict(BASE, nx=64, ny=40))
    m0, ok0 = sim.stats()
    sim.step(200)
    m1, ok1 = sim.stats()
    assert ok0 and ok1
    nodes = 64 * 40
    assert abs(m1["mass_dev"] - m0["mass_dev"]) <= 1e-13 * nodes
    assert m1["steps"] == 200


def test_step_chunking_is_invisible():
    kw = dict(BASE, nx=30, ny=10)
    a = gpu_fields(kw, 24, chunks=1)
    b = gpu_fields(kw, 24, chunks=6)
    for k in ("rho", "ux", "uy", "rho_c", "phi"):
        assert np.array_equal(a[k], b[k]), k


def test_determinism_bitwise():
    kw = dict(BASE, nx=64, ny=20)
    a = gpu_fields(kw, 30)
    b = gpu_fields(kw, 30)
    for k in ("rho", "ux", "uy", "rho_c", "phi"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("precision", ["fp64", "fp32_f64math"])
def test_launch_shapes_do_not_change_results(precision):
    """Threads per transform block, threads per collide tile and columns per
    collide tile are free to tune: the fields are bitwise the same (ny = 600
    gives two-row collide tiles; widths 64 and 37 give x-tiles with halo
    columns and a ragged last tile)."""
    from paper_1812_05711_amd.lbm_ec import Simulation
    import torch

    out = []
    for tu in ((128, 64, 1, 0), (512, 1024, 1, 0), (256, 128, 2, 0), (256, 64, 1, 64), (128, 128, 1, 37)):
        sim = Simulation(device="cuda:0", precision=precision, **dict(BASE, nx=100, ny=600))
        sim.set_tuning(*tu)
        sim.step(15)
        f = sim.fields()
        torch.cuda.synchronize()
        out.append({k: v.cpu().numpy() for k, v in f.items()})
        sim.close()
    for k in out[0]:
        for o in out[1:]:
            assert np.array_equal(out[0][k], o[k]), k
