"""The coupled time step and the nondimensional output fields.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

State after n steps: the pre-collision populations f^n and g^n, stored as
deviations from hydrostatic reference rows (see lbm.py).  One step
n -> n+1, in the order the paper's equations give it:
  1. rho_c^n = sum_i g_i^n                                 (Eq. 6)
  2. phi^n from the Poisson problem with s = -rho_c^n/eps (Eq. 4, 18-25)
  3. E^n = -grad phi^n (central differences)
  4. rho = sum f_i, F = rho_c E (+ test body force), u from Eq. 7,
     charge transport velocity v = u - mu_b grad(phi) = u + K E (Eq. 11)
  5. TRT collision of f with the source of Eq. 12 (Eq. 8, 13, 15) and of g
     (Eq. 9, 14), with the same-time-level phi^n
  6. streaming with the electrode conditions of Table I.
"""

import dataclasses

import numpy as np

from . import diagnostics, hydrostatic, lbm, poisson, splitmix
from .lattice import CI, WI, Params, lattice_constants


def round_bits(v, bits=40):
    """v rounded to `bits` significant bits (elementwise)."""
    v = np.asarray(v, dtype=np.float64)
    m, e = np.frexp(v)
    return np.ldexp(np.round(m * 2.0**bits), e - bits)


def hydrostatic_rows(p: Params, lc):
    """Lattice-unit reference rows of the closed-form state at y = j + 1/2.

    Returns (rho_c_ref, s_ref):
      rho_c_ref -- the closed-form charge profile (Eq. 27)
      s_ref     -- slope of the reference density rho_ref(y) = 1 + s_ref
                   (y - H/2), which balances the uniform closed-form force
                   density F0 = rho_c E = eps C E0 / H^3 with the lattice
                   pressure gradient: cs2 d(rho)/dy = F0, so s_ref = 3 F0.
    """
    ny = p.ny
    H = lc.H
    yj = (np.arange(ny) + 0.5) / ny
    e0 = hydrostatic.field_at_injector(p.C)
    _, rc_nd, _ = hydrostatic.profiles(p.C, yj)
    rho_c_ref = lc.eps / H**2 * rc_nd
    F0 = lc.eps * p.C * e0 / H**3
    return rho_c_ref, 3.0 * F0


def charge_noise(p: Params) -> np.ndarray:
    """xi(x, j) in [-1, 1): k-th SplitMix64 output, k = j*nx + x, seed + instance."""
    xi = splitmix.uniform_pm1(p.seed + p.instance_id, p.nx * p.ny)
    return xi.reshape(p.ny, p.nx)


def eq29_profile(x, y, Lx, Ly, amp):
    """The perturbation of Eq. 29 (section V.2) at points (x, y):

      u_x =  amp Lx sin(2 pi y / Ly) sin(2 pi x / Lx)
      u_y =  amp Ly (cos(2 pi y / Ly) - 1) cos(2 pi x / Lx)

    a single x wavenumber 2 pi / Lx, divergence-free, zero at the electrodes
    y = 0 and y = Ly; amp is the 1e-3 of Eq. 29 in the chosen velocity unit.
    """
    ux = amp * Lx * np.sin(2 * np.pi * y / Ly) * np.sin(2 * np.pi * x / Lx)
    uy = amp * Ly * (np.cos(2 * np.pi * y / Ly) - 1.0) * np.cos(2 * np.pi * x / Lx)
    return ux, uy


def eq29_velocity(p: Params, lc):
    """Eq. 29 at the nodes, in lattice velocity.

    x and y in units of the gap H (x = x_node / H, y = (j + 1/2) / H), Lx =
    nx / ny, Ly = 1, amplitude 1e-3 in units of u0 = K / H.
    """
    nx, ny = p.nx, p.ny
    x = (np.arange(nx) / ny)[None, :]
    y = ((np.arange(ny) + 0.5) / ny)[:, None]
    return eq29_profile(x, y, nx / ny, 1.0, 1e-3 * lc.u0)


class Oracle:
    def __init__(self, p: Params):
        self.p = p
        self.lc = lc = lattice_constants(p)
        nx, ny = p.nx, p.ny
        self.n = 0
        self.bx = float(p.body_force_x)
        self.pending_T = None
        rho_c_ref = self._set_reference_rows(p, lc)
        if p.init_mode == "rest":
            self.ft = np.zeros((9, ny, nx))
            self.gt = np.zeros((9, ny, nx))
            return
        rho_c0 = np.broadcast_to(rho_c_ref[:, None], (ny, nx)).copy()
        ux0 = np.zeros((ny, nx))
        uy0 = np.zeros((ny, nx))
        if p.init_mode == "noise":
            rho_c0 = rho_c0 * (1.0 + p.noise_amp * charge_noise(p))
        elif p.init_mode == "eq29":
            ux0, uy0 = eq29_velocity(p, lc)
        else:
            raise ValueError(f"unknown init_mode {p.init_mode!r}")
        _, D0, fl0 = poisson.solve_split(rho_c0, lc.eps)
        ex0, ey0 = poisson.electric_field(D0, fl0)
        rho = np.broadcast_to(self.rho_ref[:, None], (ny, nx))
        # f^0 = f^eq(rho_ref, u0), g^0 = g^eq(rho_c^0, u0 + K E^0)
        self.ft = lbm.equilibrium_deviation(np.zeros((ny, nx)), rho, ux0, uy0)
        drc0 = rho_c0 - self.r[:, None]
        self.gt = lbm.charge_equilibrium_deviation(drc0, rho_c0, ux0 + lc.K * ex0, uy0 + lc.K * ey0)

    # ---- pieces of one step -------------------------------------------------
    def macroscopic(self):
        """Steps 1-4 on the current pre-collision state."""
        lc = self.lc
        drc = lbm.charge_deviation(self.gt)
        rho_c = self.r[:, None] + drc
        phi_mean, D, phi_fluct = poisson.solve_split(rho_c, lc.eps)
        ex, ey = poisson.electric_field(D, phi_fluct)
        phi = phi_mean[:, None] + phi_fluct
        drho = lbm.density_deviation(self.ft)
        rho = self.rho_ref[:, None] + drho
        fx = rho_c * ex + self.bx
        fy = rho_c * ey
        ux, uy = lbm.velocity(self.ft, rho, fx, fy)
        return dict(rho_c=rho_c, drc=drc, phi=phi, phi_mean=phi_mean, ex=ex, ey=ey,
                    drho=drho, rho=rho, fx=fx, fy=fy, ux=ux, uy=uy)

    def collide(self, m):
        lc = self.lc
        om = lc.omega
        feq = lbm.equilibrium_deviation(m["drho"], m["rho"], m["ux"], m["uy"])
        src = lbm.forcing(m["ux"], m["uy"], m["fx"], m["fy"])
        ft_post = lbm.trt_collide(self.ft, feq, om["wp"], om["wm"], src)
        vx = m["ux"] + lc.K * m["ex"]
        vy = m["uy"] + lc.K * m["ey"]
        geq = lbm.charge_equilibrium_deviation(m["drc"], m["rho_c"], vx, vy)
        gt_post = lbm.trt_collide(self.gt, geq, om["wgp"], om["wgm"])
        return ft_post, gt_post

    def step(self, n: int = 1):
        for _ in range(n):
            m = self.macroscopic()
            ft_post, gt_post = self.collide(m)
            if self.pending_T is not None:
                ft_post, gt_post = self._continue_at(self.pending_T, ft_post, gt_post)
                self.pending_T = None
            self.ft = lbm.stream_fluid(ft_post, self.s_ref)
            self.gt = lbm.stream_charge(gt_post, self.R, self.lc.rho0)
            self.n += 1
        return self

    # ---- reference rows and continuation at another T ----------------------
    def _set_reference_rows(self, p: Params, lc):
        """Reference rows of parameters p, rounded so that w_i times them is
        exact (see lbm.py); returns the unrounded closed-form charge row."""
        ny = p.ny
        if p.init_mode == "rest":
            rho_c_ref, s_ref = np.zeros(ny), 0.0
        else:
            rho_c_ref, s_ref = hydrostatic_rows(p, lc)
        self.s_ref = 36.0 * float(round_bits(s_ref / 36.0))
        self.rho_ref = 1.0 + self.s_ref * ((np.arange(ny) + 0.5) - 0.5 * lc.H)
        q = round_bits(rho_c_ref / 36.0)
        self.r = 36.0 * q  # reference charge row
        self.R = (36.0 * WI)[:, None] * q[None, :]  # R_i(y) = w_i r(y), exact
        return rho_c_ref

    def set_T(self, T: float):
        """Continue the run at electric Rayleigh number T (the continuation of
        section V.2, where T is lowered after the vortices have formed).

        The paper does not say what carries over when T changes.  Reading:
        the change happens between the collision of the next step and its
        streaming, and the state keeps its nondimensional meaning --
          charge: the full post-collision populations are scaled by
            eps_new / eps_old, so rho_c / rho0 (rho_c in units of eps / H^2)
            and the field E are continuous;
          fluid: the departure of the post-collision populations from the
            hydrostatic state of the lattice is kept.  That state has
            rho_ref(y) and the uniform force s_ref / 3 in y; its pre-collision
            populations w_i (rho_ref - c_iy s_ref / 2) carry the momentum
            -F / 2 that makes u = 0 (Eq. 7), and the source of Eq. 12 adds F,
            so its post-collision populations are w_i (rho_ref + c_iy s_ref / 2).
        Everything derived from T (K, eps, rho0, D_c, the charge rates, the
        reference rows) is that of the new T from the streaming on.
        """
        lattice_constants(dataclasses.replace(self.p, T=float(T)))  # validates
        self.pending_T = float(T)
        return self

    def _continue_at(self, T, ft_post, gt_post):
        p_new = dataclasses.replace(self.p, T=T)
        lc_new = lattice_constants(p_new)
        scale = lc_new.eps / self.lc.eps
        R_old, s_old = self.R, self.s_ref
        self._set_reference_rows(p_new, lc_new)
        # g_new = scale (R_old + gt_post) - R_new, grouped so that the large
        # reference rows cancel first
        gt_new = scale * gt_post + (scale * R_old - self.R)[:, :, None]
        # ft is relative to w_i rho_ref(y): keeping f - w_i (rho_ref + c_iy s/2)
        # shifts it by w_i c_iy (s_new - s_old) / 2
        ft_new = ft_post + (WI * CI[:, 1])[:, None, None] * (0.5 * (self.s_ref - s_old))
        self.p, self.lc = p_new, lc_new
        return ft_new, gt_new

    def electrode_currents(self):
        """(injector, collector) currents of the current state: the charge
        that the next streaming brings in through the injector and takes out
        through the collector, in lattice units per step, summed over x.  The
        collector one is the cathode current I of the electric Nusselt number
        Ne_0 = I / I_0 (section V.2)."""
        m = self.macroscopic()
        _, gt_post = self.collide(m)
        g_post = gt_post + self.R[:, :, None]
        lower, upper = diagnostics.charge_boundary_fluxes(g_post, self.lc.rho0)
        return lower, -upper

    # ---- full populations (diagnostics and tests) --------------------------
    def full(self, ft, gt):
        """Full populations f, g from deviations of shape (9, ny, nx)."""
        f = ft + WI[:, None, None] * self.rho_ref[None, :, None]
        g = gt + self.R[:, :, None]
        return f, g

    # ---- outputs ----------------------------------------------------------
    def fields(self):
        """Nondimensional fields of the current state.

        rho: lattice density (drho = rho - rho_ref, the departure from the
        hydrostatic reference row; rho_m1 = rho - 1, the departure from the
        mean density, formed as (rho_ref - 1) + drho so that it keeps its
        own relative precision: rho_ref - 1 is exact, rho_ref being within
        a factor two of 1); u in u0 = K/H; rho_c in eps/H^2 (so rho_c = C
        at the injector); phi in the applied potential difference.
        """
        m = self.macroscopic()
        lc = self.lc
        return dict(
            rho=m["rho"],
            drho=m["drho"],
            rho_m1=(self.rho_ref - 1.0)[:, None] + m["drho"],
            ux=m["ux"] / lc.u0,
            uy=m["uy"] / lc.u0,
            rho_c=m["rho_c"] * lc.H**2 / lc.eps,
            phi=m["phi"],
        )
