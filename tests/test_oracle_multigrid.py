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
    # the coarse grid keeps >= 2 nodes per shortest wavelength ...
    assert mg.level_shapes((33, 33), (1.0, 1.0), np.pi / 4 + 1e-9)[-1] == (17, 17)
    # ... unless the grid is still too large for the direct coarsest solve
    assert mg.level_shapes((129, 129), (1.0, 1.0), 10.0, max_coarse=4096) == [
        (129, 129), (65, 65), (33, 33)]
    assert mg.level_shapes((129, 129), (1.0, 1.0), 10.0, max_coarse=100) == [
        (129, 129), (65, 65), (33, 33), (17, 17), (9, 9)]
    # 401 x 201 at 15 Hz: 2 nodes per wavelength stops at 51 x 101 (5151 > 4096 nodes),
    # so one more (under-resolved) level follows
    w = wl.random_field_2d(401, 201, 10.0, seed=2, freq_hz=15.0, src=(200, 5))
    kmax = w.omega * w.slowness.max()
    assert mg.level_shapes((201, 401), (10.0, 10.0), kmax) == [
        (201, 401), (101, 201), (51, 101), (26, 51)]


def test_smoothing_weight_per_level():
    """omega_J = 0.8 where omega*max(m)*max(h) < 2, else 0.5."""
    w = wl.grf_401x201()
    V = mg.VCycle(w.slowness, w.omega, 1.0, 0.5, w.h)
    assert [l.omega_j for l in V.levels[:-1]] == [0.8, 0.8, 0.8]
    w15 = wl.random_field_2d(401, 201, 10.0, seed=2, freq_hz=15.0, src=(200, 5))
    V15 = mg.VCycle(w15.slowness, w15.omega, 1.0, 0.5, w15.h)
    kmax = w15.omega * w15.slowness.max()
    for lev in V15.levels:
        expect = 0.8 if kmax * max(lev.spacing) < 2.0 else 0.5
        assert lev.omega_j == expect
    assert [l.omega_j for l in V15.levels[:-1]] == [0.8, 0.8, 0.5]


def test_under_resolved_levels_need_the_smaller_weight():
    """With the under-resolved level smoothed at 0.8 the cycle is a poor
    preconditioner (FGMRES stalls); with the per-level rule it converges."""
    from oracle import gmres as gm
    w = wl.random_field_2d(401, 201, 10.0, seed=2, freq_hz=15.0, src=(200, 5))
    H = op.helmholtz(w.slowness, w.omega, w.alpha, w.h)
    b = op.weighted_rhs(w.source)
    V = mg.VCycle(w.slowness, w.omega, 1.0, 0.5, w.h)
    good = gm.gmres(lambda v: H @ v, b, 1e-6, 30, 150, prec=V)
    assert good.status == gm.OK
    for lev in V.levels:
        lev.omega_j = 0.8
    bad = gm.gmres(lambda v: H @ v, b, 1e-6, 30, 150, prec=V)
    assert bad.status == gm.NOT_CONVERGED


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
    assert lev0.omega_j == 0.8
    S = np.eye(N) - lev0.omega_j * np.diag(1.0 / np.diag(M)) @ M
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


def test_three_level_cycle_uses_each_levels_weight():
    """Three levels with weights (0.8, 0.5): the cycle matrix B satisfies
    I - B M0 = S0^2 (I - P0 B1 R0 M0) S0^2 with B1 the two-grid cycle of level 1
    (its own smoother S1 = I - 0.5 D1^{-1} M1, exact coarsest solve)."""
    m = wl.smooth_slowness_2d(9, 9, 10.0, 6)
    V = mg.VCycle(m, 2 * np.pi * 3, 1.0, 0.5, 10.0)
    assert len(V.levels) == 3
    V.levels[1].omega_j = 0.5
    B = V.as_matrix()
    L0, L1, L2 = V.levels
    M0, M1, M2 = (L.M.toarray() for L in V.levels)
    I0, I1 = np.eye(M0.shape[0]), np.eye(M1.shape[0])
    S0 = I0 - 0.8 * np.diag(1 / np.diag(M0)) @ M0
    S1 = I1 - 0.5 * np.diag(1 / np.diag(M1)) @ M1
    P0, R0, P1, R1 = (x.toarray() for x in (L0.P, L0.R, L1.P, L1.R))
    E1 = S1 @ S1 @ (I1 - P1 @ sla.solve(M2, R1 @ M1)) @ S1 @ S1
    B1 = (I1 - E1) @ sla.inv(M1)
    E0 = S0 @ S0 @ (I0 - P0 @ B1 @ R0 @ M0) @ S0 @ S0
    assert np.abs((I0 - B @ M0) - E0).max() < 1e-10
