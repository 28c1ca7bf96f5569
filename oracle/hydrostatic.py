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


def steady_state_with_diffusion(C: float, Fe: float):
    """The 1-D steady state of the model equations with charge diffusion
    (section V.1 without the drift-only simplification of Eq. 27-28), the
    continuum solution the lattice hydrostatic state converges to.

    Nondimensional (gap 1, potential drop 1, eps = 1, current in units of the
    mobility): phi' = -E, E' = rho_c (Gauss), and the uniform current
    J = rho_c E - rho_c' / Fe, i.e. rho_c' = Fe (rho_c E - J); with
    phi(0) = 1, phi(1) = 0, rho_c(0) = C at the injector and rho_c'(1) = 0 at
    the collector (the zero normal gradient of Table I as read).

    Solved by shooting from the collector, where the unknowns are E(1) and J
    (then rho_c(1) = J / E(1)): integrating towards the injector the stiff
    charge mode decays, so an implicit Runge-Kutta (Radau IIA) integration at
    rtol 1e-12 is stable; Newton iteration on phi(0) = 1, rho_c(0) = C.
    Returns (J, f) with f(y) -> (E(y), rho_c(y), phi(y)) for y in [0, 1].
    """
    from scipy.integrate import solve_ivp
    from scipy.optimize import fsolve

    def rhs(y, Y, J):
        _, E, r = Y
        return [-E, r, Fe * (r * E - J)]

    def integrate(q, dense=False):
        E1, J = q
        return solve_ivp(rhs, (1.0, 0.0), [0.0, E1, J / E1], args=(J,), method="Radau", rtol=1e-12,
                         atol=1e-14, dense_output=dense)

    def miss(q):
        s = integrate(q)
        return [s.y[0, -1] - 1.0, s.y[2, -1] - C]

    import warnings

    e0 = field_at_injector(C)
    with warnings.catch_warnings():
        # the step tolerance is below what the residual allows; the residual
        # is checked below
        warnings.simplefilter("ignore", RuntimeWarning)
        q = fsolve(miss, [math.sqrt(e0 * e0 + 2.0 * C * e0), C * e0], xtol=1e-14)
    if max(abs(v) for v in miss(q)) > 1e-10:
        raise RuntimeError("shooting did not converge")
    sol = integrate(q, dense=True).sol

    def f(y):
        Y = sol(np.asarray(y, dtype=np.float64))
        return Y[1], Y[2], Y[0]

    return float(q[1]), f
