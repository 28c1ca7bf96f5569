"""D2Q9 lattice and the mapping of the physical groups onto TRT rates.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Lattice units throughout: dx = dy = dt = 1, mean fluid density 1, electrode
gap H = ny, applied potential difference 1 (phi = 1 at the lower electrode,
phi = 0 at the upper one).
"""

from dataclasses import dataclass, field

import numpy as np

# D2Q9 velocity set (section IV.2; the paper defers the table to its
# supplement, so this is the standard ordering: rest, 4 axis, 4 diagonal).
CI = np.array(
    [[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]],
    dtype=np.int64,
)
WI = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=np.float64)
# opposite direction: c_opp(i) = -c_i (the bar-i of Eq. 13-15)
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6], dtype=np.int64)
# lattice speed of sound squared (text after Eq. 12)
CS2 = 1.0 / 3.0


@dataclass
class Params:
    """Inputs of one simulation.

    nx, ny    -- grid (periodic in x; electrodes at y = 0 and y = ny)
    T, C, M, Fe -- nondimensional groups of Eq. 26
    tau_plus  -- fluid symmetric relaxation time; sets the viscosity (Eq. 16)
    Lambda, Lambda_g -- TRT "magic" products of Eq. 17 (fluid, charge)
    init_mode -- 'noise' (hydrostatic + seeded relative charge noise),
                 'eq29' (hydrostatic + the velocity perturbation of Eq. 29),
                 'rest' (rho = 1, u = 0, no charge)
    noise_amp, seed, instance_id -- charge noise amplitude and its generator key
    body_force_x -- uniform x body force (a test hook for Poiseuille flow)
    charge_rates -- which TRT rate of the charge lattice carries D_c:
                 'antisymmetric' (default): D_c = cs2 (1/w_g- - 1/2) and
                 Lambda_g sets w_g+; 'symmetric': the labels of Eq. 16 as
                 printed, D_c = cs2 (1/w_g+ - 1/2) and Lambda_g sets w_g-.
                 The diffusivity of a TRT advection-diffusion lattice is
                 carried by the antisymmetric rate, so only the default
                 gives the charge the diffusivity K / Fe.
    """

    nx: int
    ny: int
    T: float = 200.0
    C: float = 10.0
    M: float = 10.0
    Fe: float = 4000.0
    tau_plus: float = 0.8
    Lambda: float = 0.25
    Lambda_g: float = 1e-6
    init_mode: str = "noise"
    noise_amp: float = 1e-3
    seed: int = 181205711
    instance_id: int = 0
    body_force_x: float = 0.0
    charge_rates: str = "antisymmetric"


@dataclass
class LatticeConstants:
    H: float
    nu: float  # kinematic viscosity
    K: float  # ion mobility mu_b
    eps: float  # permittivity
    rho0: float  # injected charge density at the lower electrode
    Dc: float  # charge diffusivity
    tau_p: float
    tau_m: float
    tau_gp: float
    tau_gm: float
    u0: float  # velocity unit K * dphi0 / H
    t0: float  # ionic time H^2 / K
    omega: dict = field(default_factory=dict)


def lattice_constants(p: Params) -> LatticeConstants:
    """Lattice values of the physical constants.

    The paper does not print this mapping; it follows from Eq. 16-17 and the
    definitions of Eq. 26 with rho = 1, dphi0 = 1, H = ny:
      nu   = cs2 (tau+ - 1/2)                      (Eq. 16)
      T    = eps / (nu K)  and  M = sqrt(eps) / K  => K = nu T / M^2, eps = (M K)^2
      C    = rho0 H^2 / eps                        => rho0 = C eps / H^2
      Fe   = K / Dc                                => Dc = K / Fe
      Dc   = cs2 (tau_g - 1/2)                     (Eq. 16)
      Lambda = (tau+ - 1/2)(tau- - 1/2)            (Eq. 17), same for the charge.
    tau_g is the antisymmetric charge time unless p.charge_rates says
    'symmetric' (the label printed in Eq. 16); Lambda_g then fixes the other.
    """
    if not (p.tau_plus > 0.5):
        raise ValueError("tau_plus must exceed 1/2")
    if p.Lambda <= 0 or p.Lambda_g <= 0:
        raise ValueError("Lambda and Lambda_g must be positive")
    if p.nx < 1 or p.ny < 3:
        raise ValueError("grid too small")
    if not (p.T > 0 and p.M > 0 and p.Fe > 0 and p.C >= 0):
        raise ValueError("T, M, Fe must be positive and C non-negative")
    H = float(p.ny)
    nu = CS2 * (p.tau_plus - 0.5)
    K = nu * p.T / p.M**2
    eps = (p.M * K) ** 2
    rho0 = p.C * eps / H**2
    Dc = K / p.Fe
    tau_p = p.tau_plus
    tau_m = 0.5 + p.Lambda / (tau_p - 0.5)
    tau_gd = 0.5 + Dc / CS2  # carries the diffusivity
    tau_go = 0.5 + p.Lambda_g / (tau_gd - 0.5)  # set by Lambda_g
    if p.charge_rates == "antisymmetric":
        tau_gp, tau_gm = tau_go, tau_gd
    elif p.charge_rates == "symmetric":
        tau_gp, tau_gm = tau_gd, tau_go
    else:
        raise ValueError(f"unknown charge_rates {p.charge_rates!r}")
    lc = LatticeConstants(
        H=H,
        nu=nu,
        K=K,
        eps=eps,
        rho0=rho0,
        Dc=Dc,
        tau_p=tau_p,
        tau_m=tau_m,
        tau_gp=tau_gp,
        tau_gm=tau_gm,
        u0=K / H,
        t0=H * H / K,
    )
    lc.omega = {
        "wp": 1.0 / tau_p,
        "wm": 1.0 / tau_m,
        "wgp": 1.0 / tau_gp,
        "wgm": 1.0 / tau_gm,
    }
    return lc
