"""TRT lattice Boltzmann pieces of section IV.2 (Eq. 5-15) and Table I.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Storage: the fluid populations are kept as deviations
    ft_i(x, y) = f_i(x, y) - w_i rho_ref(y)
from the hydrostatic reference density rho_ref(y) = 1 + s_ref (y - H/2), a
row profile that is linear in y with slope s_ref.  This is an exact change
of variables: the collision acts on f_i - f_i^eq and on f_i^+- - f_i^eq+-,
where w_i rho_ref cancels because w_i = w_opp(i); bounce-back stays in its
row; streaming from row y - c_iy adds the known constant
w_i (rho_ref(y - c_iy) - rho_ref(y)) = -w_i c_iy s_ref.  It keeps the FP64
rounding of the small velocity field far below the round-off of f_i ~ 0.44
and of the hydrostatic pressure profile.

The charge populations are kept the same way, as gt_i(x, y) = g_i(x, y) -
R_i(y) with R_i(y) = w_i r(y) for a reference charge row r(y) (the
closed-form profile).  r is rounded to a multiple of 36 with few significant
bits, so every R_i (36 w_i is 16, 4 or 1) and every difference of R_i
between neighbouring rows is exact in FP64; with that the change of
variables is exact in floating point as well, and the nearly
non-dissipative charge lattice no longer accumulates the round-off of the
full g_i.  Arrays have shape (9, ny, nx): direction, row y, column x.
"""

import numpy as np

from .lattice import CI, WI, OPP

CX = CI[:, 0].astype(np.float64)[:, None, None]
CY = CI[:, 1].astype(np.float64)[:, None, None]
W3 = WI[:, None, None]


def density_deviation(ft):
    """rho - rho_ref = sum_i ft_i   (Eq. 5)."""
    return ft.sum(axis=0)


def charge_deviation(gt):
    """rho_c - r = sum_i gt_i   (Eq. 6 on the deviations)."""
    return gt.sum(axis=0)


def velocity(ft, rho, fx, fy):
    """u from rho u = sum_i c_i f_i + F dt / 2   (Eq. 7).

    sum_i c_i w_i = 0, so the deviations give the same first moment.
    """
    jx = (CX * ft).sum(axis=0)
    jy = (CY * ft).sum(axis=0)
    return (jx + 0.5 * fx) / rho, (jy + 0.5 * fy) / rho


def equilibrium_deviation(drho, rho, ux, uy):
    """f_i^eq - w_i rho_ref for Eq. 10 with cs2 = 1/3 and drho = rho - rho_ref:
    w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u) - w_i rho_ref
      = w_i drho + w_i rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u).
    """
    cu = CX * ux + CY * uy
    uu = ux * ux + uy * uy
    return W3 * drho + W3 * rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu)


def charge_equilibrium_deviation(drc, rho_c, vx, vy):
    """g_i^eq - R_i for Eq. 11 with cs2 = 1/3, transport velocity v and
    drc = rho_c - r:
    w_i rho_c (1 + 3 c.v + 9/2 (c.v)^2 - 3/2 v.v) - w_i r
      = w_i drc + w_i rho_c (3 c.v + 9/2 (c.v)^2 - 3/2 v.v).
    """
    cv = CX * vx + CY * vy
    vv = vx * vx + vy * vy
    return W3 * drc + W3 * rho_c * (3.0 * cv + 4.5 * cv * cv - 1.5 * vv)


def forcing(ux, uy, fx, fy):
    """F_i = w_i [ (c_i - u)/cs2 + (c_i.u) c_i / cs2^2 ] . F   (Eq. 12)."""
    cu = CX * ux + CY * uy
    ax = 3.0 * (CX - ux) + 9.0 * cu * CX
    ay = 3.0 * (CY - uy) + 9.0 * cu * CY
    return W3 * (ax * fx + ay * fy)


def sym_antisym(a):
    """(a_i + a_opp(i)) / 2 and (a_i - a_opp(i)) / 2   (Eq. 13-15)."""
    ao = a[OPP]
    return 0.5 * (a + ao), 0.5 * (a - ao)


def trt_collide(a, a_eq, w_plus, w_minus, src=None):
    """Post-collision values of Eq. 8 (with the source) or Eq. 9 (without).

    a* = a - w+ (a+ - a_eq+) - w- (a- - a_eq-) + (1 - w+/2) S+ + (1 - w-/2) S-
    """
    ap, am = sym_antisym(a)
    ep, em = sym_antisym(a_eq)
    out = a - w_plus * (ap - ep) - w_minus * (am - em)
    if src is not None:
        sp, sm = sym_antisym(src)
        out = out + (1.0 - 0.5 * w_plus) * sp + (1.0 - 0.5 * w_minus) * sm
    return out


def stream_fluid(ft_post, s_ref):
    """Pull streaming of the fluid populations with halfway bounce-back at
    both electrodes (Table I: bounce-back for f_i at the upper and lower
    walls; the walls sit half a cell outside the first and last rows).

    f_i(x, y) <- f*_i(x - c_ix, y - c_iy); a source row outside the channel
    is replaced by the node's own reflected population f*_opp(i)(x, y).
    On the deviations from w_i rho_ref(y) (slope s_ref), a population that
    changes row picks up -w_i c_iy s_ref; bounce-back stays in its row.
    """
    _, ny, nx = ft_post.shape
    out = np.empty_like(ft_post)
    for i in range(9):
        cx, cy = int(CI[i, 0]), int(CI[i, 1])
        shifted = np.roll(ft_post[i], shift=cx, axis=1)  # value from x - cx
        rebase = -WI[i] * cy * s_ref
        if cy == 0:
            out[i] = shifted
        elif cy == 1:
            out[i, 1:] = shifted[:-1] + rebase  # from row y - 1
            out[i, 0] = ft_post[OPP[i], 0]  # lower wall bounce-back
        else:
            out[i, :-1] = shifted[1:] + rebase  # from row y + 1
            out[i, ny - 1] = ft_post[OPP[i], ny - 1]  # upper wall bounce-back
    return out


def stream_charge(gt_post, R, rho0):
    """Pull streaming of the charge populations with the electrode conditions.

    Reading of Table I: its macroscopic conditions are rho_c = rho0 at the
    lower electrode (injector) and a zero normal gradient at the upper one
    (collector), and the current that Eq. 27-28 assume must leave through
    the collector.  So:
      lower wall, incoming directions (c_iy = +1): anti-bounce-back, which
        fixes the wall value rho_c = rho0:
          g_i(x, 0) = -g*_opp(i)(x, 0) + 2 w_i rho0
      upper wall, incoming directions (c_iy = -1): zero normal gradient of
        g_i (the ghost row copies the last row):
          g_i(x, ny-1) = g*_i(x - c_ix, ny-1)
    On the deviations gt = g - R (R has shape (9, ny) and R_i = R_opp(i)):
    a population arriving from row y - c_iy picks up R_i(y - c_iy) - R_i(y),
    and the injector value becomes -gt*_opp(i) + 2 (w_i rho0 - R_i(0)).
    """
    _, ny, nx = gt_post.shape
    out = np.empty_like(gt_post)
    for i in range(9):
        cx, cy = int(CI[i, 0]), int(CI[i, 1])
        shifted = np.roll(gt_post[i], shift=cx, axis=1)
        if cy == 0:
            out[i] = shifted
        elif cy == 1:
            out[i, 1:] = shifted[:-1] + (R[i, :-1] - R[i, 1:])[:, None]
            out[i, 0] = -gt_post[OPP[i], 0] + 2.0 * (WI[i] * rho0 - R[i, 0])
        else:
            out[i, :-1] = shifted[1:] + (R[i, 1:] - R[i, :-1])[:, None]
            out[i, ny - 1] = shifted[ny - 1]
    return out
