"""Pins of the oracle's lattice algebra (section IV.2, Eq. 5-17, Eq. 26).

Each check compares against mathematics the paper fixes (moment identities
of Eq. 10-12, the definitions of Eq. 16-17 and Eq. 26), never against the
oracle itself.
"""

import numpy as np
import pytest

from oracle import lbm, splitmix
from oracle.lattice import CI, CS2, OPP, WI, Params, lattice_constants


def test_splitmix64_published_vectors():
    # First outputs of SplitMix64 seeded with 1234567, as published with the
    # generator's reference implementations.
    expect = [
        6457827717110365317,
        3203168211198807973,
        9817491932198370423,
        4593380528125082431,
        16408922859458223821,
    ]
    assert [int(v) for v in splitmix.outputs(1234567, 5)] == expect
    # counter form: output k does not depend on how many were drawn before
    assert int(splitmix.outputs(1234567, 1, start=3)[0]) == expect[3]
    xi = splitmix.uniform_pm1(7, 100000)
    assert xi.min() >= -1.0 and xi.max() < 1.0
    assert abs(xi.mean()) < 0.01 and abs(xi.var() - 1.0 / 3.0) < 0.01


def test_d2q9_isotropy():
    c = CI.astype(float)
    assert np.isclose(WI.sum(), 1.0, rtol=0, atol=1e-16)
    assert np.allclose(WI @ c, 0.0, atol=1e-17)
    second = np.einsum("i,ia,ib->ab", WI, c, c)
    assert np.allclose(second, CS2 * np.eye(2), atol=1e-16)
    third = np.einsum("i,ia,ib,ic->abc", WI, c, c, c)
    assert np.allclose(third, 0.0, atol=1e-17)
    fourth = np.einsum("i,ia,ib,ic,id->abcd", WI, c, c, c, c)
    d = np.eye(2)
    iso = CS2**2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                    + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(fourth, iso, atol=1e-16)
    # opposite directions (bar-i of Eq. 13-15)
    assert np.array_equal(CI[OPP], -CI)
    assert np.array_equal(WI[OPP], WI)


@pytest.mark.parametrize("T,C,M,Fe,tau,lam,lamg,ny", [
    (200.0, 10.0, 10.0, 4000.0, 0.8, 0.25, 1e-6, 100),
    (163.4, 10.0, 10.0, 4000.0, 1.0, 1 / 12, 1e-6, 100),
    (300.0, 1.0, 7.0, 100.0, 0.65, 3 / 16, 1e-3, 840),
])
def test_parameter_mapping_reproduces_eq16_eq17_eq26(T, C, M, Fe, tau, lam, lamg, ny):
    p = Params(nx=8, ny=ny, T=T, C=C, M=M, Fe=Fe, tau_plus=tau, Lambda=lam, Lambda_g=lamg)
    lc = lattice_constants(p)
    rho, dphi, H = 1.0, 1.0, float(ny)
    mu = rho * lc.nu
    # Eq. 26, evaluated forward from the lattice constants
    assert np.isclose(np.sqrt(lc.eps / rho) / lc.K, M, rtol=1e-14)
    assert np.isclose(lc.eps * dphi / (mu * lc.K), T, rtol=1e-14)
    assert np.isclose(lc.rho0 * H**2 / (lc.eps * dphi), C, rtol=1e-14)
    assert np.isclose(lc.K * dphi / lc.Dc, Fe, rtol=1e-14)
    # Eq. 16 and Eq. 17 with dt = 1; D_c on the antisymmetric charge rate
    w = lc.omega
    assert np.isclose(CS2 * (1 / w["wp"] - 0.5), lc.nu, rtol=1e-14)
    assert np.isclose(CS2 * (1 / w["wgm"] - 0.5), lc.Dc, rtol=1e-9)
    assert np.isclose((1 / w["wp"] - 0.5) * (1 / w["wm"] - 0.5), lam, rtol=1e-13)
    assert np.isclose((1 / w["wgp"] - 0.5) * (1 / w["wgm"] - 0.5), lamg, rtol=1e-9)
    # the labels of Eq. 16 as printed
    p.charge_rates = "symmetric"
    w2 = lattice_constants(p).omega
    assert np.isclose(CS2 * (1 / w2["wgp"] - 0.5), lc.Dc, rtol=1e-9)
    assert np.isclose(w2["wgp"], w["wgm"]) and np.isclose(w2["wgm"], w["wgp"])


def test_parameter_validation():
    with pytest.raises(ValueError):
        lattice_constants(Params(nx=8, ny=8, tau_plus=0.5))
    with pytest.raises(ValueError):
        lattice_constants(Params(nx=8, ny=2))
    with pytest.raises(ValueError):
        lattice_constants(Params(nx=8, ny=8, Lambda=0.0))


def _random_state(seed, shape=(5, 7)):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.01 * rng.standard_normal(shape)
    ux = 0.02 * rng.standard_normal(shape)
    uy = 0.02 * rng.standard_normal(shape)
    fx = 1e-3 * rng.standard_normal(shape)
    fy = 1e-3 * rng.standard_normal(shape)
    return rho, ux, uy, fx, fy


def test_equilibrium_moments():
    """Eq. 10: zeroth, first and second moments of f^eq."""
    rho, ux, uy, _, _ = _random_state(1)
    rho_ref = 1.0 + 0.003 * np.arange(rho.shape[0])[:, None] * np.ones_like(rho)
    dev = lbm.equilibrium_deviation(rho - rho_ref, rho, ux, uy)
    feq = dev + WI[:, None, None] * rho_ref[None]
    c = CI.astype(float)
    assert np.allclose(feq.sum(0), rho, rtol=0, atol=1e-15)
    assert np.allclose(np.einsum("i,i...->...", c[:, 0], feq), rho * ux, atol=1e-16)
    assert np.allclose(np.einsum("i,i...->...", c[:, 1], feq), rho * uy, atol=1e-16)
    pxx = np.einsum("i,i...->...", c[:, 0] ** 2, feq)
    pxy = np.einsum("i,i...->...", c[:, 0] * c[:, 1], feq)
    pyy = np.einsum("i,i...->...", c[:, 1] ** 2, feq)
    assert np.allclose(pxx, rho * CS2 + rho * ux * ux, atol=1e-15)
    assert np.allclose(pxy, rho * ux * uy, atol=1e-16)
    assert np.allclose(pyy, rho * CS2 + rho * uy * uy, atol=1e-15)


def test_charge_equilibrium_moments():
    """Eq. 11: sum g^eq = rho_c and sum c g^eq = rho_c (u - mu_b grad phi)."""
    rho, vx, vy, _, _ = _random_state(2)
    rc = 4e-3 * rho
    r = 3.9e-3 * np.ones(rho.shape[0])
    R = WI[:, None] * r[None, :]
    g = lbm.charge_equilibrium_deviation(rc - r[:, None], rc, vx, vy) + R[:, :, None]
    c = CI.astype(float)
    assert np.allclose(g.sum(0), rc, rtol=1e-14, atol=0)
    assert np.allclose(np.einsum("i,i...->...", c[:, 0], g), rc * vx, rtol=1e-13)
    assert np.allclose(np.einsum("i,i...->...", c[:, 1], g), rc * vy, rtol=1e-13)


def test_forcing_moments():
    """Eq. 12: sum F_i = 0, sum c_i F_i = F, sum c_i c_i F_i = uF + Fu."""
    _, ux, uy, fx, fy = _random_state(3)
    F = lbm.forcing(ux, uy, fx, fy)
    c = CI.astype(float)
    assert np.allclose(F.sum(0), 0.0, atol=1e-18)
    assert np.allclose(np.einsum("i,i...->...", c[:, 0], F), fx, atol=1e-18)
    assert np.allclose(np.einsum("i,i...->...", c[:, 1], F), fy, atol=1e-18)
    assert np.allclose(np.einsum("i,i...->...", c[:, 0] ** 2, F), 2 * ux * fx, atol=1e-18)
    assert np.allclose(np.einsum("i,i...->...", c[:, 0] * c[:, 1], F), ux * fy + uy * fx, atol=1e-18)


def test_trt_split_and_collision_invariants():
    """Eq. 8, 13, 15: the +/- parts rebuild the populations; the collision with
    the source conserves mass and adds exactly F dt to the momentum once the
    half-force velocity of Eq. 7 is used."""
    rng = np.random.default_rng(4)
    shape = (4, 6)
    rho_ref = np.ones(shape[0])
    ft = 1e-3 * rng.standard_normal((9,) + shape)
    ap, am = lbm.sym_antisym(ft)
    assert np.allclose(ap + am, ft, atol=1e-19)
    assert np.allclose(ap[OPP], ap) and np.allclose(am[OPP], -am)
    fx = 1e-4 * rng.standard_normal(shape)
    fy = 1e-4 * rng.standard_normal(shape)
    drho = lbm.density_deviation(ft)
    rho = rho_ref[:, None] + drho
    ux, uy = lbm.velocity(ft, rho, fx, fy)
    feq = lbm.equilibrium_deviation(drho, rho, ux, uy)
    src = lbm.forcing(ux, uy, fx, fy)
    for wp, wm in [(1.25, 0.75), (1.9, 1.1), (1.0, 1.0)]:
        post = lbm.trt_collide(ft, feq, wp, wm, src)
        c = CI.astype(float)
        assert np.allclose(post.sum(0), ft.sum(0), atol=1e-18)
        jx0 = np.einsum("i,i...->...", c[:, 0], ft)
        jy0 = np.einsum("i,i...->...", c[:, 1], ft)
        jx1 = np.einsum("i,i...->...", c[:, 0], post)
        jy1 = np.einsum("i,i...->...", c[:, 1], post)
        assert np.allclose(jx1 - jx0, fx, atol=1e-17)
        assert np.allclose(jy1 - jy0, fy, atol=1e-17)
    # charge: no source, conserves rho_c for any rates
    gt = 1e-4 * rng.standard_normal((9,) + shape)
    geq = lbm.charge_equilibrium_deviation(gt.sum(0), 4e-3 + gt.sum(0), ux, uy)
    gpost = lbm.trt_collide(gt, geq, 1.9994, 1.97)
    assert np.allclose(gpost.sum(0), gt.sum(0), atol=1e-19)
