"""Pins of the oracle's discrete operator and direct solve (CPU only).

Each test checks the oracle against something it does not compute itself:
dense LU, closed-form lattice and continuous Green's functions, manufactured
solutions of the continuous boundary-value problem (Eq. 2 with the
first-order absorbing boundary), polynomial exactness and symmetry.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.special as ssp

from oracle import operator as op
from oracle import direct
import workloads as wl


def _het_2d(nz, nx, h=10.0, seed=0):
    return wl.smooth_slowness_2d(nz, nx, h, seed)


# --------------------------------------------------------------------------
# structure
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(33,), (9, 11), (7, 5)])
def test_exactly_complex_symmetric(shape):
    m = wl.smooth_slowness_2d(1, shape[0], 10.0, 1)[0] if len(shape) == 1 else _het_2d(*shape)
    for sigma in (1 - 0.01j, 1 - 0.5j, 0.0, -1 + 0.3j):
        A = op.assemble(m, 2 * np.pi * 12.0, sigma, 10.0).toarray()
        assert np.array_equal(A, A.T)


def test_shift_one_alpha_is_helmholtz():
    m = _het_2d(9, 11)
    H = op.helmholtz(m, 60.0, 0.01, 10.0)
    M = op.shifted_laplace(m, 60.0, 1.0, 0.01, 10.0)
    assert abs(H - M).max() == 0.0


def test_zero_shift_interior_rows_are_negative_laplacian():
    """At zero shift the interior rows are the 5-point -Lap_h: exact on quadratics."""
    nz, nx, hz, hx = 9, 13, 7.0, 3.0
    m = _het_2d(nz, nx)
    A = op.assemble(m, 40.0, 0.0, (hz, hx))
    z = np.arange(nz)[:, None] * hz
    x = np.arange(nx)[None, :] * hx
    for u, lap in ((x ** 2 + z ** 2, 4.0), (3 * x ** 2 - z ** 2 + x * z, 4.0), (x + 2 * z, 0.0)):
        out = (A @ u.ravel().astype(complex)).reshape(nz, nx)
        assert np.allclose(out[1:-1, 1:-1], -lap, atol=1e-9)
    n, h = 17, 4.0
    A1 = op.assemble(np.full(n, 1 / 2000.0), 40.0, 0.0, h)
    x = np.arange(n) * h
    out = A1 @ (x ** 2).astype(complex)
    assert np.allclose(out[1:-1], -2.0, atol=1e-9)


# --------------------------------------------------------------------------
# manufactured solutions: second-order convergence including the absorbing
# boundary rows, their 1/2 and 1/4 weights and the sign of the boundary term
# --------------------------------------------------------------------------
def _mms_2d(nz, nx, Lz=0.8, Lx=1.0, alpha=0.05, omega=6.0):
    hz, hx = Lz / (nz - 1), Lx / (nx - 1)
    z = np.arange(nz)[:, None] * hz
    x = np.arange(nx)[None, :] * hx
    c = 1.0 + 0.3 * np.sin(2.0 * x) * np.cos(3.0 * z)
    m = 1.0 / c
    k = omega * m
    sigma = 1 - 1j * alpha
    a, b, x0, z0, s = 4.0, -3.0, 0.45, 0.35, 0.5
    phi = -1j * (a * x + b * z) - ((x - x0) ** 2 + (z - z0) ** 2) / s ** 2
    u = np.exp(phi)
    px = -1j * a - 2 * (x - x0) / s ** 2
    pz = -1j * b - 2 * (z - z0) / s ** 2
    lap = (-2 / s ** 2 + px ** 2 - 2 / s ** 2 + pz ** 2) * u
    f = -lap - sigma * k ** 2 * u
    # inhomogeneous first-order ABC data g = du/dn + j k u on each face;
    # a centred ghost point turns it into a source 2 g / h on the face nodes
    F = f.copy()
    F[:, 0] += 2 / hx * (-(px * u) + 1j * k * u)[:, 0]
    F[:, -1] += 2 / hx * ((px * u) + 1j * k * u)[:, -1]
    F[0, :] += 2 / hz * (-(pz * u) + 1j * k * u)[0, :]
    F[-1, :] += 2 / hz * ((pz * u) + 1j * k * u)[-1, :]
    A = op.assemble(m, omega, sigma, (hz, hx))
    uh = direct.solve_matrix(A, op.weighted_rhs(F)).reshape(nz, nx)
    return np.abs(uh - u).max() / np.abs(u).max()


def test_manufactured_2d_second_order():
    errs = [_mms_2d(1 + 8 * r, 1 + 10 * r) for r in (2, 4, 8)]
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert errs[-1] < 2e-3
    for q in ratios:
        assert 3.5 < q < 4.6, (errs, ratios)


def _mms_1d(n, L=1.0, alpha=0.05, omega=7.0):
    h = L / (n - 1)
    x = np.arange(n) * h
    m = 1.0 / (1.0 + 0.4 * np.sin(3.0 * x))
    k = omega * m
    sigma = 1 - 1j * alpha
    a, x0, s = 5.0, 0.4, 0.6
    u = np.exp(-1j * a * x - (x - x0) ** 2 / s ** 2)
    px = -1j * a - 2 * (x - x0) / s ** 2
    f = -(-2 / s ** 2 + px ** 2) * u - sigma * k ** 2 * u
    F = f.copy()
    F[0] += 2 / h * (-px[0] * u[0] + 1j * k[0] * u[0])
    F[-1] += 2 / h * (px[-1] * u[-1] + 1j * k[-1] * u[-1])
    A = op.assemble(m, omega, sigma, h)
    uh = direct.solve_matrix(A, op.weighted_rhs(F))
    return np.abs(uh - u).max() / np.abs(u).max()


def test_manufactured_1d_second_order():
    errs = [_mms_1d(1 + 20 * r) for r in (1, 2, 4, 8)]
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    for q in ratios:
        assert 3.7 < q < 4.3, (errs, ratios)


# --------------------------------------------------------------------------
# 1D homogeneous lattice: exact finite-lattice closed form
# --------------------------------------------------------------------------
def test_1d_lattice_closed_form():
    n, h, c, freq, alpha, s = 1001, 5.0, 2000.0, 10.0, 0.01, 100
    omega = 2 * np.pi * freq
    k = omega / c
    kt2 = (1 - 1j * alpha) * k ** 2
    # root |xi| < 1 of xi^2 - (2 - kt2 h^2) xi + 1 = 0
    roots = np.roots([1.0, -(2.0 - kt2 * h * h), 1.0])
    xi = roots[np.argmin(np.abs(roots))]
    assert abs(xi) < 1

    i = np.arange(n)

    def left(i):   # u_i = a1 xi^i + b1 xi^(s-i), valid for i <= s (and its ghost i=-1)
        return np.array([xi ** i, xi ** (s - i), 0 * i, 0 * i], dtype=complex)

    def right(i):  # u_i = a2 xi^(i-s) + b2 xi^(n-1-i), valid for i >= s (and ghost i=n)
        return np.array([0 * i, 0 * i, xi ** (i - s), xi ** (n - 1 - i)], dtype=complex)

    rows, rhs = [], []
    rows.append(left(s) - right(s)); rhs.append(0.0)               # continuity at s
    # centred ABC at each end: -(u_1 - u_-1)/(2h) + j k u_0 = 0, (u_n - u_{n-2})/(2h) + j k u_{n-1} = 0
    rows.append(-(left(1) - left(-1)) / (2 * h) + 1j * k * left(0)); rhs.append(0.0)
    rows.append((right(n) - right(n - 2)) / (2 * h) + 1j * k * right(n - 1)); rhs.append(0.0)
    # source row: (2u_s - u_{s-1} - u_{s+1})/h^2 - kt2 u_s = 1
    rows.append((2 * left(s) - left(s - 1) - right(s + 1)) / h ** 2 - kt2 * left(s)); rhs.append(1.0)
    coef = np.linalg.solve(np.array(rows), np.array(rhs, dtype=complex))
    exact = np.where(i <= s, coef[0] * xi ** i + coef[1] * xi ** (s - i),
                     coef[2] * xi ** (i - s) + coef[3] * xi ** (n - 1 - i))

    m = np.full(n, 1.0 / c)
    u = direct.solve_direct(m, omega, alpha, h, wl.point_source((n,), s))
    assert np.abs(u - exact).max() / np.abs(exact).max() < 1e-11


def test_1d_continuous_green_function_second_order():
    """Lossless homogeneous 1D: the first-order ABC is exact for the outgoing
    Green's function G = exp(-j k |x - s|)/(2 j k); a unit nodal source is a
    delta of weight h, so u -> h G at second order."""
    L, c, freq = 2000.0, 2000.0, 10.0
    omega = 2 * np.pi * freq
    k = omega / c
    errs = []
    for h in (10.0, 5.0, 2.5):
        n = int(round(L / h)) + 1
        s = (n - 1) // 4
        x = np.arange(n) * h
        u = direct.solve_direct(np.full(n, 1 / c), omega, 0.0, h, wl.point_source((n,), s))
        G = h * np.exp(-1j * k * np.abs(x - x[s])) / (2j * k)
        errs.append(np.abs(u - G).max() / np.abs(G).max())
    # the error is the accumulated phase (dispersion) error, k L (k h)^2 / 24
    assert errs[-1] < 1.5e-2
    for a, b in zip(errs, errs[1:]):
        assert 3.6 < a / b < 4.4, errs


def test_2d_point_source_matches_hankel():
    """Damped homogeneous 2D medium: u -> h^2 G with G = (-j/4) H0^(2)(kt r), the
    outgoing Green's function for exp(+j w t), at second order in h (fixed
    physical ring around the source, away from the faces)."""
    c, freq, alpha, L = 2000.0, 20.0, 0.25, 800.0
    omega = 2 * np.pi * freq
    kt = (omega / c) * np.sqrt(1 - 1j * alpha)
    errs = []
    for h in (5.0, 2.5):
        n = int(round(L / h)) + 1
        s = (n // 2, n // 2)
        u = direct.solve_direct(np.full((n, n), 1 / c), omega, alpha, h,
                                wl.point_source((n, n), s))
        iz, ix = np.mgrid[0:n, 0:n]
        r = h * np.hypot(iz - s[0], ix - s[1])
        ring = (r > 80.0) & (r < 150.0)
        G = -0.25j * ssp.hankel2(0, kt * r[ring])
        errs.append((np.abs(u[ring] / h ** 2 - G) / np.abs(G)).max())
    assert errs[-1] < 0.012, errs
    assert errs[0] / errs[1] > 3.0, errs


# --------------------------------------------------------------------------
# direct solve and reciprocity
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(64,), (9, 11), (7, 5)])
def test_splu_matches_dense_lu(shape):
    if len(shape) == 1:
        m = 1.0 / wl.layered_velocity_1d(shape[0], 5.0)
    else:
        m = _het_2d(*shape)
    f = wl.random_complex(shape, 3)
    u = direct.solve_direct(m, 2 * np.pi * 10, 0.01, 10.0, f)
    H = op.helmholtz(m, 2 * np.pi * 10, 0.01, 10.0).toarray()
    ud = sla.solve(H, op.weighted_rhs(f)).reshape(shape)
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 1e-12


def test_reciprocity():
    nz, nx = 31, 41
    m = _het_2d(nz, nx, seed=5)
    omega = 2 * np.pi * 15
    s, r = (7, 9), (20, 33)
    us = direct.solve_direct(m, omega, 0.01, 10.0, wl.point_source((nz, nx), s))
    ur = direct.solve_direct(m, omega, 0.01, 10.0, wl.point_source((nz, nx), r))
    assert abs(us[r] - ur[s]) / abs(us[r]) < 1e-10
