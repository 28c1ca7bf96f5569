"""Fast Poisson solve for the electric potential (section IV.3, Eq. 18-25).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Discrete problem (Eq. 18): [D_x^2 + D_y^2] phi = s with s = -rho_c / eps
(Eq. 4), D_x^2 spectral in the periodic x direction (Eq. 19-20) and D_y^2 the
3-point second difference in y (the symbol of Eq. 24).

Geometry reading: nodes sit at y = j + 1/2 (j = 0 .. ny-1) and the electrodes
at y = 0 and y = ny, so the Dirichlet values are imposed through ghost nodes:
    phi(-1) = 2 phi_lower - phi(0),     phi(ny) = 2 phi_upper - phi(ny-1)
with phi_lower = 1 and phi_upper = 0.  The paper's odd extension (Eq. 21-22)
with the shift of Eq. 23 diagonalises exactly this operator when the
extension is taken about the half-cell wall positions; for each x wavenumber
it is the tridiagonal system below, which is what this oracle solves.

For each x wavenumber m (after the forward DFT of Eq. 19):
    phi_m(j+1) - (2 + kappa_m^2) phi_m(j) + phi_m(j-1) = s_m(j)
with kappa_m = 2 pi min(m, nx-m) / nx (Eq. 20, wavenumbers folded into the
Nyquist band) and the ghosts above, whose non-zero Dirichlet value enters the
m = 0 right-hand side as -2 * DFT(1) = -2 nx.  The inverse DFT carries the
1/nx normalisation.
"""

import numpy as np


def wavenumbers(nx: int) -> np.ndarray:
    """kappa_m for m = 0 .. nx-1 (Eq. 20 with folded indices)."""
    m = np.arange(nx)
    return 2.0 * np.pi * np.minimum(m, nx - m) / nx


def dft_x(a: np.ndarray) -> np.ndarray:
    """Eq. 19 along the last axis: forward, unnormalised."""
    return np.fft.fft(a, axis=-1)


def idft_x(a_hat: np.ndarray) -> np.ndarray:
    """Inverse of Eq. 19 along the last axis, with the 1/nx factor."""
    return np.fft.ifft(a_hat, axis=-1)


def thomas(sub, diag, sup, rhs):
    """Tridiagonal elimination (Thomas algorithm) along axis 0.

    sub[j] x[j-1] + diag[j] x[j] + sup[j] x[j+1] = rhs[j]; arrays of shape
    (n, ...) solved independently for every trailing index.
    """
    n = rhs.shape[0]
    cp = np.empty(diag.shape, dtype=np.result_type(diag, sup))
    dp = np.empty(rhs.shape, dtype=np.result_type(rhs, diag))
    cp[0] = sup[0] / diag[0]
    dp[0] = rhs[0] / diag[0]
    for j in range(1, n):
        den = diag[j] - sub[j] * cp[j - 1]
        cp[j] = sup[j] / den
        dp[j] = (rhs[j] - sub[j] * dp[j - 1]) / den
    x = np.empty_like(dp)
    x[n - 1] = dp[n - 1]
    for j in range(n - 2, -1, -1):
        x[j] = dp[j] - cp[j] * x[j + 1]
    return x


def solve_spectral_rhs(s_hat: np.ndarray, nx: int, phi_lower: float = 1.0, phi_upper: float = 0.0):
    """Solve every wavenumber's y system; s_hat has shape (ny, nx) complex."""
    ny = s_hat.shape[0]
    kappa2 = wavenumbers(nx) ** 2
    diag = np.empty((ny, nx))
    diag[:] = -(2.0 + kappa2)
    # ghost closures: phi(-1) = 2 phi_lower - phi(0) and phi(ny) = 2 phi_upper - phi(ny-1)
    diag[0] -= 1.0
    diag[ny - 1] -= 1.0
    rhs = s_hat.astype(np.complex128).copy()
    rhs[0, 0] -= 2.0 * phi_lower * nx  # DFT of the constant boundary value at m = 0
    rhs[ny - 1, 0] -= 2.0 * phi_upper * nx
    ones = np.ones((ny, nx))
    return thomas(ones, diag, ones, rhs)


def solve_split(rho_c: np.ndarray, eps: float, phi_lower: float = 1.0, phi_upper: float = 0.0):
    """The potential as (x-mean row, fluctuation) from the charge density.

    phi(x, y) = phi_mean(y) + phi_fluct(x, y), where phi_mean comes from the
    m = 0 mode alone and phi_fluct from the m >= 1 modes.  Keeping the two
    apart is an exact identity; it stops the O(1) rounding of phi from
    swamping the small transverse field that the fluctuation carries.
    """
    ny, nx = rho_c.shape
    s = -rho_c / eps  # Eq. 4
    s_hat = dft_x(s)  # Eq. 19
    phi_hat = solve_spectral_rhs(s_hat, nx, phi_lower, phi_upper)  # Eq. 20, 24-25
    phi_mean = phi_hat[:, 0].real / nx
    fl = phi_hat.copy()
    fl[:, 0] = 0.0
    phi_fluct = idft_x(fl).real
    return phi_mean, phi_fluct


def solve(rho_c: np.ndarray, eps: float, phi_lower: float = 1.0, phi_upper: float = 0.0):
    """phi on the (ny, nx) node grid from the charge density (Eq. 4, 18-25)."""
    phi_mean, phi_fluct = solve_split(rho_c, eps, phi_lower, phi_upper)
    return phi_mean[:, None] + phi_fluct


def electric_field(phi_mean: np.ndarray, phi_fluct: np.ndarray,
                   phi_lower: float = 1.0, phi_upper: float = 0.0):
    """E = -grad(phi) by second-order central differences.

    The paper does not state how the gradient for the force (Eq. 7, 12) and
    the drift (Eq. 11) is formed; this uses central differences, periodic in
    x, with the same ghost values at the electrodes as the Poisson solve.
    The mean row and the fluctuation are differenced separately (the ghost
    rule is linear, so the mean row takes the Dirichlet values and the
    fluctuation takes zero).
    """
    ny, nx = phi_fluct.shape
    mean_ext = np.empty(ny + 2)
    mean_ext[1:-1] = phi_mean
    mean_ext[0] = 2.0 * phi_lower - phi_mean[0]
    mean_ext[-1] = 2.0 * phi_upper - phi_mean[-1]
    fl_ext = np.empty((ny + 2, nx))
    fl_ext[1:-1] = phi_fluct
    fl_ext[0] = -phi_fluct[0]
    fl_ext[-1] = -phi_fluct[-1]
    ey = -(mean_ext[2:] - mean_ext[:-2])[:, None] / 2.0 - (fl_ext[2:] - fl_ext[:-2]) / 2.0
    ex = -(np.roll(phi_fluct, -1, axis=1) - np.roll(phi_fluct, 1, axis=1)) / 2.0
    return ex, ey
