"""Pins of the oracle's Poisson solve (section IV.3, Eq. 18-25).

 - Eq. 19 against the textbook O(N^2) DFT sum;
 - the tridiagonal elimination against a dense LAPACK solve;
 - a discrete manufactured solution: the test applies the discrete operator
   (exact spectral x-derivative of a cosine, 3-point y-stencil with the
   electrode ghosts) forward and checks that the solver inverts it;
 - the paper's own route (odd extension in y, FFT, division by the symbol of
   Eq. 25), built in the test from Eq. 21-25 with the extension taken about
   the half-cell wall positions, agrees with the tridiagonal;
 - a smooth continuous solution converges at second order (section IV.4);
 - a charge-free channel has the uniform field 1/H at every row.
"""

import numpy as np
import pytest

from oracle import poisson


def test_dft_matches_textbook_sum():
    rng = np.random.default_rng(11)
    for nx in (1, 2, 5, 12, 61, 122):
        a = rng.standard_normal((3, nx))
        x = np.arange(nx)
        k = np.arange(nx)
        kernel = np.exp(-2j * np.pi * np.outer(x, k) / nx)  # Eq. 19, 0-based
        ref = a @ kernel
        assert np.allclose(poisson.dft_x(a), ref, rtol=0, atol=1e-12 * nx)
        back = poisson.idft_x(ref)
        assert np.allclose(back.real, a, atol=1e-13)


def test_thomas_matches_dense_solve():
    rng = np.random.default_rng(12)
    n, m = 40, 5
    sub = rng.uniform(0.5, 1.0, (n, m))
    sup = rng.uniform(0.5, 1.0, (n, m))
    diag = -(2.5 + rng.uniform(0, 1, (n, m)))
    rhs = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    x = poisson.thomas(sub, diag, sup, rhs)
    for c in range(m):
        A = np.diag(diag[:, c]) + np.diag(sub[1:, c], -1) + np.diag(sup[:-1, c], 1)
        ref = np.linalg.solve(A, rhs[:, c])
        assert np.allclose(x[:, c], ref, rtol=1e-13, atol=1e-13)


def _apply_discrete_operator(phi_of_y, kx, nx, phi_lower, phi_upper):
    """[D_x^2 + D_y^2] of phi(x, y) = A(y) + B(y) cos(2 pi kx x / nx).

    D_x^2 is spectral (Eq. 20), so it multiplies the cosine by -kappa^2; D_y^2
    is the 3-point stencil with ghost nodes mirroring the electrode values.
    """
    A, B = phi_of_y
    ny = A.size
    kap2 = (2 * np.pi * min(kx, nx - kx) / nx) ** 2

    def d2y(v, lo, hi):
        ext = np.concatenate([[2 * lo - v[0]], v, [2 * hi - v[-1]]])
        return ext[2:] - 2 * ext[1:-1] + ext[:-2]

    x = np.arange(nx)
    cos = np.cos(2 * np.pi * kx * x / nx)
    sA = d2y(A, phi_lower, phi_upper)
    sB = d2y(B, 0.0, 0.0) - kap2 * B
    phi = A[:, None] + B[:, None] * cos[None, :]
    s = sA[:, None] + sB[:, None] * cos[None, :]
    return phi, s


@pytest.mark.parametrize("nx,ny,kx", [(16, 12, 3), (122, 100, 1), (61, 9, 30), (8, 3, 4)])
def test_manufactured_discrete_solution(nx, ny, kx):
    rng = np.random.default_rng(13)
    A = rng.standard_normal(ny)
    B = rng.standard_normal(ny)
    phi_star, s = _apply_discrete_operator((A, B), kx, nx, 1.0, 0.0)
    eps = 2.5
    rho_c = -s * eps
    phi = poisson.solve(rho_c, eps)
    assert np.max(np.abs(phi - phi_star)) < 1e-12 * max(1.0, np.max(np.abs(phi_star)))
    mean, D, fl = poisson.solve_split(rho_c, eps)
    assert np.allclose(mean, A, atol=1e-12)
    ext = np.concatenate([[2.0 - A[0]], A, [-A[-1]]])
    assert np.allclose(D, ext[1:] - ext[:-1], atol=1e-12)
    assert np.allclose(fl, B[:, None] * np.cos(2 * np.pi * kx * np.arange(nx) / nx)[None, :],
                       atol=1e-12)


@pytest.mark.parametrize("ny", [3, 10, 100, 840])
def test_mean_mode_flux_form_matches_dense_solve(ny):
    """The m = 0 solve in flux form equals a dense LAPACK solve of the same
    3-point system with the electrode ghosts."""
    rng = np.random.default_rng(15)
    sbar = -1e-3 * (1.0 + rng.uniform(0, 1, ny))
    A = -2.0 * np.eye(ny) + np.eye(ny, k=1) + np.eye(ny, k=-1)
    A[0, 0] = A[-1, -1] = -3.0
    rhs = sbar.copy()
    rhs[0] -= 2.0 * 1.0
    ref = np.linalg.solve(A, rhs)
    mean, D = poisson.mean_mode(sbar, 1.0, 0.0)
    # the dense solve's own error grows with the condition number ~ ny^2
    assert np.max(np.abs(mean - ref)) < 1e-15 * max(ny * ny, 100)
    ext = np.concatenate([[2.0 - ref[0]], ref, [-ref[-1]]])
    assert np.allclose(D, ext[1:] - ext[:-1], rtol=1e-9, atol=1e-13)


def test_odd_extension_route_of_eq21_25():
    """Solve the same problem the paper's way: subtract the boundary lift,
    extend the source oddly in y about the walls (length 2 ny), 2-D FFT,
    divide by -(k_x^2 + 4 sin^2(k_y / 2)) (Eq. 25), inverse FFT, keep the
    first half."""
    rng = np.random.default_rng(14)
    nx, ny = 24, 20
    s = rng.standard_normal((ny, nx))
    eps = 1.0
    phi = poisson.solve(-s * eps, eps)
    # lift: the discrete linear profile with phi = 1 / 0 at the walls has zero
    # second difference, including the ghost rows
    yj = np.arange(ny) + 0.5
    lift = 1.0 - yj / ny
    ext = np.concatenate([s, -s[::-1]], axis=0)  # odd about the half-cell walls
    hat = np.fft.fft2(ext)
    kx = 2 * np.pi * np.minimum(np.arange(nx), nx - np.arange(nx)) / nx
    ky = 2 * np.pi * np.arange(2 * ny) / (2 * ny)
    symbol = -(kx[None, :] ** 2 + 4 * np.sin(ky[:, None] / 2) ** 2)
    symbol[0, 0] = 1.0  # the (0,0) mode of an odd extension is zero
    psi = np.fft.ifft2(hat / symbol).real[:ny]
    assert np.max(np.abs(phi - (lift[:, None] + psi))) < 1e-12


def test_second_order_convergence_to_continuous_solution():
    """phi = (1 - y) + sin(pi y) cos(2 pi x / Lx) on [0, Lx] x [0, 1]."""
    errs = []
    for ny in (16, 32, 64):
        nx = 2 * ny
        Lx = nx / ny
        x = np.arange(nx) / ny
        y = (np.arange(ny) + 0.5) / ny
        X, Y = np.meshgrid(x, y)
        exact = (1 - Y) + np.sin(np.pi * Y) * np.cos(2 * np.pi * X / Lx)
        lap = -(np.pi**2 + (2 * np.pi / Lx) ** 2) * np.sin(np.pi * Y) * np.cos(2 * np.pi * X / Lx)
        # lattice units: dx = 1 = H / ny, so the source scales by 1 / ny^2
        s = lap / ny**2
        phi = poisson.solve(-s, 1.0)
        errs.append(np.max(np.abs(phi - exact)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs


def test_uniform_field_without_charge():
    nx, ny = 10, 7
    mean, D, fl = poisson.solve_split(np.zeros((ny, nx)), 3.0)
    ex, ey = poisson.electric_field(D, fl)
    assert np.allclose(ey, 1.0 / ny, rtol=1e-13)
    assert np.allclose(ex, 0.0, atol=1e-17)
    assert np.allclose(mean, 1.0 - (np.arange(ny) + 0.5) / ny, atol=1e-14)


def test_field_of_a_transverse_mode():
    """E = -grad phi by central differences of a known potential."""
    nx, ny = 32, 16
    A = np.linspace(1, 0, ny)
    B = np.sin(np.pi * (np.arange(ny) + 0.5) / ny)
    x = np.arange(nx)
    fl = B[:, None] * np.cos(2 * np.pi * x / nx)[None, :]
    extA = np.concatenate([[2.0 - A[0]], A, [-A[-1]]])
    ex, ey = poisson.electric_field(extA[1:] - extA[:-1], fl)
    ex_ref = -B[:, None] * (np.cos(2 * np.pi * (x + 1) / nx) - np.cos(2 * np.pi * (x - 1) / nx))[None, :] / 2
    assert np.allclose(ex, ex_ref, atol=1e-15)
    full = A[:, None] + fl
    ext = np.vstack([2 - full[0], full, -full[-1]])
    assert np.allclose(ey, -(ext[2:] - ext[:-2]) / 2, atol=1e-15)
