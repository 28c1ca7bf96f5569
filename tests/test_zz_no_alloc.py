"""lbm_ec_poisson_static, the Poisson solve that allocates no device memory
(its scratch is a static array of the library), against lbm_ec_poisson on an
instance of the same parameters: bit for bit, on two calls in a row with the
second on a smaller grid (the scratch keeps the first call's contents), in
FP64 and FP32 storage, and a grid too large for the scratch is refused."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

BASE = dict(T=200.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8, Lambda=0.25, Lambda_g=1e-6, noise_amp=1e-3,
            seed=181205711)


def _charge(nx, ny, seed):
    """A seeded nondimensional charge field: the injector level C times a
    decaying profile with relative noise."""
    rng = np.random.default_rng(seed)
    y = (np.arange(ny) + 0.5) / ny
    return 10.0 * np.exp(-3.0 * y)[:, None] * (1.0 + 0.3 * rng.standard_normal((ny, nx)))


def _reference(kw, rc):
    """lbm_ec_poisson on an instance (its own workspace)."""
    import torch

    from paper_1812_05711_amd.lbm_ec import Simulation

    sim = Simulation(device="cuda:0", **kw)
    phi = sim.poisson(torch.from_numpy(rc).to("cuda:0"))
    torch.cuda.synchronize()
    out = phi.cpu().numpy()
    sim.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32_f64math"])
def test_static_poisson_matches_the_instance_call(precision):
    import torch

    from paper_1812_05711_amd.lbm_ec import poisson_static

    # two calls in a row, the second smaller; then the first grid again
    cases = [(300, 260, 1), (122, 100, 2), (300, 260, 3)]
    for nx, ny, seed in cases:
        kw = dict(BASE, nx=nx, ny=ny, precision=precision)
        rc = _charge(nx, ny, seed)
        print("static poisson", precision, nx, ny, seed, flush=True)
        d_rc = torch.from_numpy(rc).to("cuda:0")
        out = torch.empty_like(d_rc)
        got = poisson_static(d_rc, out=out, **kw)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        ref = _reference(kw, rc)
        assert np.array_equal(got.cpu().numpy(), ref), (precision, nx, ny)


def test_static_poisson_refuses_a_grid_beyond_its_scratch():
    import torch

    from paper_1812_05711_amd.lbm_ec import EINVAL, STATIC_SCRATCH_BYTES, LbmEcError, poisson_static, \
        poisson_static_bytes

    kw = dict(BASE, nx=2048, ny=2048, precision="fp64")
    assert poisson_static_bytes(**kw) > STATIC_SCRATCH_BYTES
    rc = torch.zeros((2048, 2048), dtype=torch.float64, device="cuda:0")
    with pytest.raises(LbmEcError) as e:
        poisson_static(rc, **kw)
    assert e.value.code == EINVAL
    small = dict(BASE, nx=64, ny=40, precision="fp64")
    assert 0 < poisson_static_bytes(**small) <= STATIC_SCRATCH_BYTES
