"""Pins of the oracle's V-cycle (CPU only).

Checks against facts fixed by the definition and by multigrid theory rather
than by re-running the oracle: exactness of (bi)linear interpolation, the
full-weighting numbers, the known Galerkin coarse stencil of the 5-point
Laplacian, the two-grid error-propagation operator assembled from dense
factors, textbook V-cycle convergence on a definite problem, and the level
layout of the benchmark grids.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import multigrid as mg
from oracle import operator as op
import workloads as wl


def test_level_shapes_of_workload_grids():
    w = wl.grf_401x201()
    kmax = w.omega * w.slowness.max()
    assert mg.level_shapes((201, 401), (10.0, 10.0), kmax) == [
        (201, 401), (101, 201), (51, 101), (26, 51)]
    # odd (n-1) stops a dimension; (n-1)/2 >= 2 keeps at least 3 nodes
    assert mg.level_shapes((9, 9), (1.0, 1.0), 1e-3) == [(9, 9), (5, 5), (3, 3)]
    assert mg.level_shapes((17, 9), (1.0, 1.0), 1e-3) == [(17, 9), (9, 5), (5, 3), (3, 3)]
    assert mg.level_shapes((8, 9), (1.0, 1.0), 1e-3) == [(8, 9), (8, 5), (8, 3)]
    # the coarse grid keeps >= 2 nodes per shortest wavelength
    assert mg.level_shapes((33, 33), (1.0, 1.0), np.pi / 4 + 1e-9)[-1] == (17, 17)


@pytest.mark.parametrize("fine,halved", [((9, 11), (True, True)), ((9, 8), (True, False)),
                                          ((8, 9), (False, True)), ((17,), (True,))])
def test_prolongation_exact_on_multilinear(fine, halved):
    P = mg.prolongation(fine, halved)
    coarse = tuple((n - 1) // 2 + 1 if hv else n for n, hv in zip(fine, halved))
    grids_f = np.meshgrid(*[np.arange(n, dtype=float) for n in fine], indexing="ij")
    grids_c = np.meshgrid(*[np.arange(n, dtype=float) * (2 if hv else 1)
                            for n, hv in zip(coarse, halved)], indexing="ij")

    def func(g):
        if len(g) == 1:
            return 2.0 + 0.5 * g[0]
        # linear in every halved axis (any function along an untouched axis)
        za, xa = g
        return (1.0 + 0.3 * za + 0.7 * xa - 0.2 * za * xa) * (1 + 0 * za)

    uf = P @ func(grids_c).ravel()
    assert np.allclose(uf, func(grids_f).ravel(), atol=1e-13)


def test_restriction_is_full_weighting():
    fine, halved = (9, 11), (True, True)
    R = mg.restriction(fine, halved).toarray()
    P = mg.prolongation(fine, halved).toarray()
    assert np.array_equal(R, P.T / 4.0)
    # interior coarse node (I, J) = (2, 2) sits on fine node (4, 4)
    nc_x = 6
    row = R[2 * nc_x + 2].reshape(fine)
    expect = np.zeros(fine)
    expect[3:6, 3:6] = np.array([[1, 2, 1], [2, 4, 2], [1, 2, 1]]) / 16.0
    assert np.array_equal(row, expect)
    R1 = mg.restriction((9, 8), (True, False)).toarray()
    assert np.array_equal(R1, mg.prolongation((9, 8), (True, False)).toarray().T / 2.0)


def test_galerkin_coarse_stencil_of_laplacian():
    """R (-Lap_h) P with bilinear P and full weighting is the 9-point stencil
    [[-1/4,-1/2,-1/4],[-1/2,3,-1/2],[-1/4,-1/2,-1/4]] / H^2, H = 2h."""
    n, h = 17, 3.0
    V = mg.VCycle(np.full((n, n), 1e-9), 1e-6, 0.0, 0.0, h)   # k ~ 0: pure -Lap_h + tiny ABC
    Ac = V.levels[1].M.toarray()
    nc = V.levels[1].shape[1]
    I = 4 * nc + 4
    row = Ac[I].reshape(V.levels[1].shape)[3:6, 3:6]
    H = 2 * h
    expect = np.array([[-0.25, -0.5, -0.25], [-0.5, 3.0, -0.5], [-0.25, -0.5, -0.25]]) / H ** 2
    assert np.allclose(row, expect, rtol=1e-12, atol=1e-15)


def test_galerkin_operators_complex_symmetric():
    V = mg.VCycle(wl.smooth_slowness_2d(17, 33, 10.0, 2), 2 * np.pi * 5, 1.0, 0.5, 10.0)
    assert len(V.levels) >= 3
    for lev in V.levels:
        A = lev.M.toarray()
        assert np.allclose(A, A.T, rtol=0, atol=1e-14 * np.abs(A).max())


def test_jacobi_fixed_point():
    V = mg.VCycle(wl.smooth_slowness_2d(9, 11, 10.0, 2), 2 * np.pi * 5, 1.0, 0.5, 10.0)
    lev = V.levels[0]
    x = wl.random_complex(lev.M.shape[0], 1)
    assert np.allclose(V.jacobi(lev, x, lev.M @ x), x, rtol=1e-14, atol=0)


def test_two_grid_error_propagation():
    """With two levels, I - B M = S^2 (I - P Mc^{-1} R M) S^2, S = I - w D^{-1} M."""
    m = wl.smooth_slowness_2d(9, 9, 10.0, 4)
    V = mg.VCycle(m, 2 * np.pi * 4, 1.0, 0.5, 10.0)
    V.levels = V.levels[:2]
    lev0, lev1 = V.levels
    import scipy.sparse.linalg as spla
    lev1.lu = spla.splu(lev1.M.tocsc())
    B = V.as_matrix()
    M = lev0.M.toarray()
    N = M.shape[0]
    S = np.eye(N) - 0.8 * np.diag(1.0 / np.diag(M)) @ M
    P = lev0.P.toarray()
    R = lev0.R.toarray()
    Mc = R @ M @ P
    E = S @ S @ (np.eye(N) - P @ sla.solve(Mc, R @ M)) @ S @ S
    assert np.abs((np.eye(N) - B @ M) - E).max() < 1e-11


def test_single_level_is_exact_inverse():
    m = wl.smooth_slowness_2d(8, 8, 10.0, 3)            # n-1 = 7 is odd: no coarsening
    V = mg.VCycle(m, 2 * np.pi * 4, 1.0, 0.5, 10.0)
    assert len(V.levels) == 1
    M = op.shifted_laplace(m, 2 * np.pi * 4, 1.0, 0.5, 10.0).toarray()
    assert np.abs(V.as_matrix() @ M - np.eye(64)).max() < 1e-11


def test_vcycle_converges_on_definite_problem():
    """Textbook behaviour: V(2,2) omega-Jacobi multigrid as a stationary iteration
    on a definite (positively shifted) operator converges fast and
    independently of h."""
    rates = []
    for n in (33, 65):
        h = 640.0 / (n - 1)
        m = np.full((n, n), 1 / 2000.0)
        omega = 2 * np.pi * 2.0
        V = mg.VCycle(m, omega, -1.0, 0.0, h)           # M = -Lap + k^2 (+ ABC)
        M = V.levels[0].M
        b = wl.random_complex(n * n, 7)
        x = np.zeros_like(b)
        r0 = np.linalg.norm(b)
        for _ in range(8):
            x = x + V(b - M @ x)
        rates.append((np.linalg.norm(b - M @ x) / r0) ** (1 / 8))
    assert max(rates) < 0.15, rates
    assert abs(rates[0] - rates[1]) < 0.05, rates
