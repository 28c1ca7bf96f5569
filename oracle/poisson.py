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


def mean_mode(sbar: np.ndarray, phi_lower: float = 1.0, phi_upper: float = 0.0):
    """The x-mean (m = 0) part of the Poisson problem, by integrating Gauss's
    law twice.

    With D(j) = phi(j+1) - phi(j) for j = -1 .. ny-1 (the ghost rows
    included), the 3-point equation of row j reads D(j) - D(j-1) = sbar(j),
    so D(j) = D(-1) + S(j) with S the running sum of sbar.  The ghost rules
    give D(-1) = 2 (phi(0) - phi_lower) and D(ny-1) = 2 (phi_upper -
    phi(ny-1)); eliminating phi(0) yields
        D(-1) = (phi_upper - phi_lower) / ny - (S(ny-1) + 2 sum_{k<ny-1} S(k)) / (2 ny)
    with no cancellation.  This is the same tridiagonal system the other
    modes solve; the flux form keeps the round-off of the mean field at the
    level of the sums instead of the O(1) potential.

    Returns (phi_mean of length ny, D of length ny + 1 holding D(-1) .. D(ny-1)).
    """
    ny = sbar.size
    S = np.cumsum(sbar)
    T = S[: ny - 1].sum()
    d_lower = (phi_upper - phi_lower) / ny - (S[ny - 1] + 2.0 * T) / (2.0 * ny)
    D = np.concatenate([[d_lower], d_lower + S])
    phi0 = phi_lower + 0.5 * d_lower
    phi_mean = phi0 + np.concatenate([[0.0], np.cumsum(D[1:ny])])
    return phi_mean, D


def solve_split(rho_c: np.ndarray, eps: float, phi_lower: float = 1.0, phi_upper: float = 0.0):
    """The potential as x-mean row and fluctuation from the charge density.

    phi(x, y) = phi_mean(y) + phi_fluct(x, y), where phi_mean comes from the
    m = 0 mode (solved in flux form by mean_mode) and phi_fluct from the
    m >= 1 modes (tridiagonal per mode).  Keeping the two apart is an exact
    identity; it stops the O(1) rounding of phi from swamping the small
    fields that the transverse modes and the mean flux carry.

    Returns (phi_mean, D, phi_fluct); D are the mean-row differences of
    mean_mode.
    """
    ny, nx = rho_c.shape
    s = -rho_c / eps  # Eq. 4
    s_hat = dft_x(s)  # Eq. 19
    phi_mean, D = mean_mode(s_hat[:, 0].real / nx, phi_lower, phi_upper)
    fl_hat = s_hat.copy()
    fl_hat[:, 0] = 0.0
    # m >= 1: homogeneous Dirichlet ghosts (the boundary values live in m = 0)
    phi_hat = solve_spectral_rhs(fl_hat, nx, 0.0, 0.0)  # Eq. 20, 24-25
    phi_hat[:, 0] = 0.0
    phi_fluct = idft_x(phi_hat).real
    return phi_mean, D, phi_fluct


def solve(rho_c: np.ndarray, eps: float, phi_lower: float = 1.0, phi_upper: float = 0.0):
    """phi on the (ny, nx) node grid from the charge density (Eq. 4, 18-25)."""
    phi_mean, _, phi_fluct = solve_split(rho_c, eps, phi_lower, phi_upper)
    return phi_mean[:, None] + phi_fluct


def electric_field(D: np.ndarray, phi_fluct: np.ndarray):
    """E = -grad(phi) by second-order central differences.

    The paper does not state how the gradient for the force (Eq. 7, 12) and
    the drift (Eq. 11) is formed; this uses central differences, periodic in
    x, with the same ghost values at the electrodes as the Poisson solve.
    The mean row enters through its differences D (mean_mode):
    -(phi(j+1) - phi(j-1)) / 2 = -(D(j) + D(j-1)) / 2; the fluctuation has
    zero ghost values (phi_fluct(-1) = -phi_fluct(0), likewise at the top).
    """
    ny, nx = phi_fluct.shape
    fl_ext = np.empty((ny + 2, nx))
    fl_ext[1:-1] = phi_fluct
    fl_ext[0] = -phi_fluct[0]
    fl_ext[-1] = -phi_fluct[-1]
    ey_mean = -(D[1:] + D[:-1]) / 2.0
    ey = ey_mean[:, None] - (fl_ext[2:] - fl_ext[:-2]) / 2.0
    ex = -(np.roll(phi_fluct, -1, axis=1) - np.roll(phi_fluct, 1, axis=1)) / 2.0
    return ex, ey
