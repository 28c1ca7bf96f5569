"""Closed-form hydrostatic state between the electrodes (section V.1).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Without diffusion and without flow, charge conservation makes the current
rho_c * E uniform, and Gauss's law dE/dy = rho_c (nondimensional, eps = 1,
gap 1, potential drop 1) then gives E^2 linear in y.  That is the form of
Eq. 27-28:  rho_c = rho_a (y + y_a)^(-1/2),  E = 2 rho_a (y + y_a)^(1/2).
With rho_c(0) = C at the injector and integral_0^1 E dy = 1 (the applied
potential drop) one writes it through the field at the injector E0:

    E(y)     = sqrt(E0^2 + 2 C E0 y)
    rho_c(y) = C E0 / E(y)
    phi(y)   = 1 - [(E0^2 + 2 C E0 y)^(3/2) - E0^3] / (3 C E0)

so that rho_a = sqrt(C E0 / 2) and y_a = E0 / (2 C), and E0 is the root of
    [(E0^2 + 2 C E0)^(3/2) - E0^3] / (3 C E0) = 1.
"""

import math

import numpy as np


def field_at_injector(C: float) -> float:
    """E0 > 0 solving the potential-drop condition, by FP64 bisection to 1 ulp."""
    if C == 0.0:
        return 1.0  # uniform field, no space charge

    def drop(e0):
        return ((e0 * e0 + 2.0 * C * e0) ** 1.5 - e0**3) / (3.0 * C * e0) - 1.0

    lo, hi = 0.0, 1.0  # drop(0+) = -1 < 0 and drop(1) >= 0
    while True:
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if drop(mid) < 0.0:
            lo = mid
        else:
            hi = mid
    return hi


def analytic_parameters(C: float):
    """(rho_a, y_a) of Eq. 27-28 in nondimensional units."""
    e0 = field_at_injector(C)
    return math.sqrt(C * e0 / 2.0), e0 / (2.0 * C)


def profiles(C: float, y: np.ndarray):
    """Nondimensional E(y), rho_c(y), phi(y) at positions y in [0, 1]."""
    e0 = field_at_injector(C)
    y = np.asarray(y, dtype=np.float64)
    if C == 0.0:
        return np.full_like(y, 1.0), np.zeros_like(y), 1.0 - y
    e2 = e0 * e0 + 2.0 * C * e0 * y
    E = np.sqrt(e2)
    rho_c = C * e0 / E
    phi = 1.0 - (e2**1.5 - e0**3) / (3.0 * C * e0)
    return E, rho_c, phi
