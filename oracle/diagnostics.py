"""Diagnostics and error norms.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""

import numpy as np

from .lattice import CI, WI


def total_mass_deviation(ft):
    """sum over nodes of (rho - 1)."""
    return float(ft.sum())


def total_charge(g):
    return float(g.sum())


def charge_boundary_fluxes(g_post, rho0):
    """Charge that streaming the post-collision g* moves across each
    electrode in one step: (in through the lower one, net in through the
    upper one).

    Lower electrode (injector): each outgoing g*_i (c_iy = -1) is replaced
    by the anti-bounce-back value -g*_i + 2 w_i rho0 in the opposite
    direction.  Upper electrode (collector): outgoing directions (c_iy = +1)
    leave the channel and the incoming ones (c_iy = -1) copy the last row.
    """
    down = CI[:, 1] == -1
    up = CI[:, 1] == 1
    lower = np.sum(2.0 * WI[down][:, None] * rho0 - 2.0 * g_post[down, 0, :])
    upper = np.sum(g_post[down, -1, :]) - np.sum(g_post[up, -1, :])
    return float(lower), float(upper)


def charge_boundary_change(g_post, rho0):
    """Net charge that streaming adds in one step.  Collision conserves
    sum_i g_i, so Q^{n+1} - Q^n equals this."""
    lower, upper = charge_boundary_fluxes(g_post, rho0)
    return lower + upper


def rel_max_error(x, ref):
    """max |x - ref| / max |ref|  (0 when both vanish)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref))
    num = np.max(np.abs(x - ref))
    if den == 0.0:
        return float(num)
    return float(num / den)


def rel_l2_error(x, ref):
    """sqrt(sum (x - ref)^2 / sum ref^2): the e_L2 norm of Table II (read as
    relative L2, the paper does not print its definition)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.sqrt(np.sum((x - ref) ** 2) / np.sum(ref**2)))
