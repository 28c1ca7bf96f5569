"""Pins of the oracle's continuation at another T and of its electrode
currents (section V.2: Ne_0 = I / I_0 with the cathode current I, and T
lowered after the vortices have formed).

The reading being pinned (the paper is silent on it): the change takes effect
between a collision and the next streaming; the full charge populations are
scaled by eps_new / eps_old, and the fluid populations keep their departure
from the hydrostatic state of the lattice.  The pins state its consequences
on the moments, which the oracle never computes from that statement:
  * rho_c scales by eps_new / eps_old exactly, so rho_c / rho0 and E are
    continuous;
  * Eq. 7 (rho u = sum c f + F / 2) then fixes the momentum change of one
    step exactly, at every row (the wall rows included);
  * a change to the same T changes nothing, bit for bit.
The electrode currents are pinned by charge conservation (injector and
collector currents equal at steady state) and by the closed-form hydrostatic
current of Eq. 27-28 (drift only): the current density K rho_c E is uniform,
C e0 in units of K (eps / H^2) / H, so a column carries eps K C e0 / H^3.
"""

import copy

import numpy as np
import pytest

from oracle import Oracle, Params, hydrostatic


def _pair(T2, steps=10, cls=Oracle, **kw):
    """Two runs from the same state: one more step at T = 200 (a) and one
    step across a change to T2 (b)."""
    base = dict(nx=4, ny=24, T=200.0, noise_amp=1e-3)
    base.update(kw)
    a = cls(Params(**base))
    a.step(steps)
    b = copy.deepcopy(a)
    a.step(1)
    b.set_T(T2)
    b.step(1)
    return a, b


def test_change_to_the_same_T_changes_nothing():
    a, b = _pair(200.0)
    assert np.array_equal(a.ft, b.ft) and np.array_equal(a.gt, b.gt)
    assert b.p.T == 200.0 and b.pending_T is None


@pytest.mark.parametrize("T2", [150.0, 260.0])
def test_charge_keeps_its_nondimensional_value(T2):
    a, b = _pair(T2)
    scale = b.lc.eps / a.lc.eps
    assert scale == pytest.approx((T2 / 200.0) ** 2, rel=1e-14)
    ma, mb = a.macroscopic(), b.macroscopic()
    np.testing.assert_allclose(mb["rho_c"], scale * ma["rho_c"], rtol=1e-13, atol=0)
    emax = np.abs(ma["ey"]).max()
    np.testing.assert_allclose(mb["ex"], ma["ex"], rtol=0, atol=1e-12 * emax)
    np.testing.assert_allclose(mb["ey"], ma["ey"], rtol=0, atol=1e-12 * emax)
    fa, fb = a.fields(), b.fields()
    np.testing.assert_allclose(fb["rho_c"], fa["rho_c"], rtol=1e-13, atol=0)


def _momentum_residual(a, b):
    """Eq. 7 across the change, at every node: with the departure from the
    hydrostatic state kept, the streamed populations of run b differ from
    those of run a by -w_i c_iy (s_new - s_old) / 2, so
      rho_b u_b - rho_a u_a = -(s_new - s_old) / 6 y-hat + (scale - 1) F_a / 2
    (rho_c scales, E is continuous, no body force).  Returns the largest
    residual of the two components and the size of the s term."""
    scale = b.lc.eps / a.lc.eps
    ma, mb = a.macroscopic(), b.macroscopic()
    ds = b.s_ref - a.s_ref
    rx = mb["rho"] * mb["ux"] - ma["rho"] * ma["ux"] - (scale - 1.0) * ma["fx"] / 2.0
    ry = mb["rho"] * mb["uy"] - ma["rho"] * ma["uy"] - (-ds / 6.0 + (scale - 1.0) * ma["fy"] / 2.0)
    return max(np.abs(rx).max(), np.abs(ry).max()), abs(ds) / 6.0


@pytest.mark.parametrize("T2", [150.0, 260.0])
def test_fluid_keeps_its_departure_from_the_hydrostatic_state(T2):
    a, b = _pair(T2)
    res, term = _momentum_residual(a, b)
    assert term > 1e-5  # the reference force really changes
    assert res <= 1e-9 * term, (res, term)


class _DroppedShift(Oracle):
    """A planted mistake: the fluid deviations are kept relative to w_i rho_ref
    (the half-force term of the hydrostatic state forgotten)."""

    def _continue_at(self, T, ft_post, gt_post):
        _, gt_new = super()._continue_at(T, ft_post, gt_post)
        return ft_post, gt_new


def test_momentum_pin_catches_a_dropped_shift():
    a, b = _pair(150.0, cls=_DroppedShift)
    res, term = _momentum_residual(a, b)
    assert res > 0.5 * term


def test_refused_T_leaves_the_run_unchanged():
    p = Params(nx=4, ny=12)
    o = Oracle(p)
    with pytest.raises(ValueError):
        o.set_T(-1.0)
    assert o.pending_T is None and o.p.T == 200.0


@pytest.mark.parametrize("ny,steps,tol", [(24, 12000, 0.05), (36, 24000, 0.01)])
def test_hydrostatic_collector_current(ny, steps, tol):
    """An x-uniform run without noise relaxes to the discrete hydrostatic
    state (about four ionic times here); its collector current is the I_0 of
    Ne_0.  Against the closed form, within the resolution of the injection
    layer (the closed form also leaves out diffusion, 1 / Fe)."""
    p = Params(nx=2, ny=ny, T=200.0, noise_amp=0.0)
    o = Oracle(p)
    o.step(steps)
    inj, col = o.electrode_currents()
    lc = o.lc
    closed = p.nx * p.C * hydrostatic.field_at_injector(p.C) * lc.eps * lc.K / lc.H**3
    assert abs(inj / col - 1.0) < 2e-3, (inj, col)
    assert abs(col / closed - 1.0) < tol, col / closed
