"""Pin of the Eq. 29 perturbation (section V.2) that starts the threshold
runs, checked against what the equation fixes rather than against a retyped
copy of it:

 - no slip: both components vanish on the electrodes y = 0 and y = Ly;
 - mass: the field is divergence-free; on the node grid the central-
   difference divergence is an O(h^2) truncation error (ratio about 4 per
   grid doubling);
 - amplitudes: max |u_x| = 1e-3 u0 Lx and max |u_y| = 2e-3 u0 Ly (the
   factor 2 from cos - 1), u0 = K / H the velocity unit of the oracle;
 - one x wavenumber 2 pi / Lx with Lx = nx / ny: on the nodes all of the
   x spectrum of each row sits in the modes +-1.

A mistake planted in the oracle's Eq. 29 (a sign, the u0 or Lx factor, the
wavenumber, the wall term) must break at least one of these; the second
test plants each in turn.
"""

import numpy as np
import pytest

import oracle.solver as solver
from oracle import Params, lattice_constants


def _nodes(nx, ny, T=190.0):
    p = Params(nx=nx, ny=ny, T=T, init_mode="eq29")
    lc = lattice_constants(p)
    ux, uy = solver.eq29_velocity(p, lc)
    return p, lc, ux, uy


def _divergence(ux, uy):
    """Central-difference divergence in units of H (node spacing 1/ny),
    periodic in x, on the interior rows."""
    ny = ux.shape[0]
    h = 1.0 / ny
    dudx = (np.roll(ux, -1, axis=1) - np.roll(ux, 1, axis=1)) / (2 * h)
    dvdy = (uy[2:] - uy[:-2]) / (2 * h)
    return dudx[1:-1] + dvdy, np.max(np.abs(dudx))


def violations():
    """Names of the Eq. 29 properties that the oracle's field breaks."""
    bad = []
    # walls: the profile itself on y = 0 and y = Ly, dense in x
    x = np.linspace(0.0, 1.22, 397)[None, :]
    amp = 1e-3
    for y in (0.0, 1.0):
        ux, uy = solver.eq29_profile(x, np.full((1, 1), y), 1.22, 1.0, amp)
        if np.max(np.abs(ux)) > 1e-15 or np.max(np.abs(uy)) > 1e-15:
            bad.append(f"wall y={y}")
    # the node fields at two resolutions, Lx / Ly = 1.22
    e = []
    for nx, ny in ((61, 50), (122, 100)):
        p, lc, ux, uy = _nodes(nx, ny)
        div, scale = _divergence(ux, uy)
        e.append(np.max(np.abs(div)) / scale)
        Lx = nx / ny
        # amplitudes: the node grid misses the extrema by O(h^2)
        if not np.isclose(np.max(np.abs(ux)), 1e-3 * lc.u0 * Lx, rtol=3e-3):
            bad.append(f"max|u_x| at {nx}x{ny}")
        if not np.isclose(np.max(np.abs(uy)), 2e-3 * lc.u0 * 1.0, rtol=3e-3):
            bad.append(f"max|u_y| at {nx}x{ny}")
        # one x wavenumber: modes +-1 of the row spectra (x = i / ny spans Lx)
        for u in (ux, uy):
            s = np.abs(np.fft.fft(u, axis=1)) ** 2
            if s[:, [1, nx - 1]].sum() < (1 - 1e-12) * s.sum():
                bad.append(f"x wavenumber at {nx}x{ny}")
                break
        # extrapolated to the walls from the first / last two rows: O(h^2)
        for u in (ux, uy):
            w0 = 1.5 * u[0] - 0.5 * u[1]
            w1 = 1.5 * u[-1] - 0.5 * u[-2]
            if max(np.max(np.abs(w0)), np.max(np.abs(w1))) > 20.0 / ny**2 * np.max(np.abs(u)):
                bad.append(f"wall extrapolation at {nx}x{ny}")
                break
    if not (e[1] < 1e-2 and 3.5 < e[0] / e[1] < 4.5):
        bad.append(f"divergence {e[0]:.3e} -> {e[1]:.3e}")
    return bad


def test_eq29_properties():
    assert violations() == []


_real = solver.eq29_profile


def _sign_uy(x, y, Lx, Ly, amp):
    ux, uy = _real(x, y, Lx, Ly, amp)
    return ux, -uy


def _no_lx(x, y, Lx, Ly, amp):
    ux, uy = _real(x, y, Lx, Ly, amp)
    return ux / Lx, uy


def _no_u0(x, y, Lx, Ly, amp):
    # the amplitude 1e-3 left in lattice units (u0 dropped)
    return _real(x, y, Lx, Ly, 1e-3)


def _double_k(x, y, Lx, Ly, amp):
    return _real(x, y, Lx / 2, Ly, amp)


def _wall_plus(x, y, Lx, Ly, amp):
    ux, uy = _real(x, y, Lx, Ly, amp)
    return ux, uy + 2.0 * amp * Ly * np.cos(2 * np.pi * x / Lx)


def _cos_ux(x, y, Lx, Ly, amp):
    ux, uy = _real(x, y, Lx, Ly, amp)
    return amp * Lx * np.cos(2 * np.pi * y / Ly) * np.sin(2 * np.pi * x / Lx), uy


@pytest.mark.parametrize("mutant", [_sign_uy, _no_lx, _no_u0, _double_k, _wall_plus, _cos_ux],
                         ids=["sign_uy", "no_Lx", "no_u0", "double_k", "wall_term", "cos_ux"])
def test_planted_mistakes_break_the_pin(monkeypatch, mutant):
    monkeypatch.setattr(solver, "eq29_profile", mutant)
    assert violations() != []
