"""Pins of the continuum steady state with diffusion (the reference of the
convergence study) and the 2nd-order convergence of the lattice hydrostatic
state towards it (the accuracy the paper states in section IV.4, whose error
analysis sits in its missing supplement).

The reference is pinned by the closed form of Eq. 27-28 (its Fe -> infinity
limit, which it approaches as 1/Fe with the current raised by diffusion),
and by Gauss's law and the potential drop integrated independently of the
ODE solver; the oracle's lattice state at ny = 24 and 48 then pins the
order."""

import numpy as np
import pytest

from oracle import Oracle, Params, hydrostatic
from oracle.diagnostics import rel_l2_error


@pytest.mark.parametrize("C", [0.1, 10.0])
def test_reference_tends_to_the_closed_form_as_one_over_Fe(C):
    J0 = C * hydrostatic.field_at_injector(C)  # drift-only current of Eq. 27-28
    Ja, fa = hydrostatic.steady_state_with_diffusion(C, 4000.0)
    Jb, fb = hydrostatic.steady_state_with_diffusion(C, 200000.0)
    # diffusion down the charge gradient adds current
    assert Ja > Jb > J0
    # 1 / Fe to leading order: a 50-fold larger Fe leaves a 50-fold smaller
    # excess (42.9 at C = 10, where the injection layer is steep)
    assert 35.0 < (Ja - J0) / (Jb - J0) < 55.0
    y = np.linspace(0.05, 0.95, 19)  # away from the boundary layers
    E, rc, phi = hydrostatic.profiles(C, y)
    Eb, rcb, phib = fb(y)
    assert np.abs(Eb - E).max() < 1e-3 * np.abs(E).max()
    assert np.abs(rcb - rc).max() < 2e-2 * np.abs(rc).max()


@pytest.mark.parametrize("C", [0.1, 10.0])
def test_reference_satisfies_gauss_and_the_potential_drop(C):
    J, f = hydrostatic.steady_state_with_diffusion(C, 4000.0)
    y = np.linspace(0.0, 1.0, 400001)
    E, rc, phi = f(y)
    trap = lambda v: float(np.sum(0.5 * (v[1:] + v[:-1]) * np.diff(y)))
    assert trap(E) == pytest.approx(1.0, abs=1e-8)             # phi(0) - phi(1)
    assert E[-1] - E[0] == pytest.approx(trap(rc), rel=1e-7)   # Gauss
    assert rc[0] == pytest.approx(C, rel=1e-10) and phi[-1] == pytest.approx(0.0, abs=1e-10)
    # the current at the collector, where rho_c' = 0, is drift alone
    assert rc[-1] * E[-1] == pytest.approx(J, rel=1e-9)


def _lattice_state(C, ny):
    p = Params(nx=1, ny=ny, T=1200.0, C=C, M=10.0, Fe=4000.0, tau_plus=1.0, Lambda=0.25, Lambda_g=1e-6,
               noise_amp=0.0)
    o = Oracle(p)
    o.step(int(4 * o.lc.t0))
    m = o.macroscopic()
    return m["ey"][:, 0] * ny, m["rho_c"][:, 0] * ny**2 / o.lc.eps


def test_lattice_hydrostatic_state_converges_at_second_order():
    _, f = hydrostatic.steady_state_with_diffusion(0.1, 4000.0)
    err = {}
    for ny in (24, 48):
        y = (np.arange(ny) + 0.5) / ny
        E, rc, _ = f(y)
        ey, rcl = _lattice_state(0.1, ny)
        err[ny] = (rel_l2_error(ey, E), rel_l2_error(rcl, rc))
    for k in range(2):
        assert 3.6 < err[24][k] / err[48][k] < 4.4, err
    assert err[48][1] < 5e-3, err
