"""Pins of the oracle's (flexible) GMRES and of the whole oracle solve (CPU only).

References used: SciPy's GMRES (an independent implementation; its per-step
residual estimate equals ours when no preconditioner is involved, and right
preconditioning is GMRES on the explicit product ``H B``), dense LU, finite
termination, the Arnoldi relation, and the paper's qualitative claims
(Section "Example", Fig. 2-4).
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import gmres as gm
from oracle import operator as op
from oracle import solver, direct, multigrid as mg, spectrum
import workloads as wl


def _scipy_history(A, b, restart, n_iter):
    hist = []
    spla.gmres(A, b, rtol=1e-15, atol=0.0, restart=restart, maxiter=n_iter // restart,
               callback=lambda pr: hist.append(pr), callback_type="pr_norm")
    return np.array(hist)


def test_unpreconditioned_history_matches_scipy():
    m = wl.smooth_slowness_2d(15, 17, 10.0, 2)
    H = op.helmholtz(m, 2 * np.pi * 8, 0.01, 10.0)
    b = op.weighted_rhs(wl.random_complex((15, 17), 4))
    res = gm.gmres(lambda v: H @ v, b, tol=1e-15, restart=10, maxiter=30, prec=None)
    ref = _scipy_history(H, b, 10, 30)
    assert len(res.history) == 31 and len(ref) == 30
    assert np.allclose(res.history[1:], ref, rtol=1e-8, atol=0)


@pytest.mark.parametrize("kind", ["exact", "mg"])
def test_right_preconditioned_history_is_gmres_on_product(kind):
    """Right preconditioning leaves the residual b - H x unchanged, so the
    estimates equal those of plain GMRES on the explicit matrix H B."""
    if kind == "exact":
        m = 1.0 / wl.layered_velocity_1d(120, 5.0)
        shape, h, freq = (120,), 5.0, 12.0
    else:
        m = wl.smooth_slowness_2d(9, 17, 10.0, 6)
        shape, h, freq = (9, 17), 10.0, 6.0
    omega = 2 * np.pi * freq
    H = op.helmholtz(m, omega, 0.01, h)
    prec = solver.make_preconditioner(m, omega, 1.0, 0.5, h, kind)
    if kind == "exact":
        B = sla.inv(op.shifted_laplace(m, omega, 1.0, 0.5, h).toarray())
    else:
        assert len(prec.levels) >= 2
        B = prec.as_matrix()
    HB = H.toarray() @ B
    b = op.weighted_rhs(wl.random_complex(shape, 9))
    for flexible in (True, False):
        res = gm.gmres(lambda v: H @ v, b, tol=1e-15, restart=8, maxiter=24, prec=prec,
                       flexible=flexible)
        ref = _scipy_history(HB, b, 8, 24)
        keep = ref > 1e-10                  # below that both are at rounding level
        assert keep.sum() >= 8
        assert np.allclose(np.array(res.history[1:])[: len(ref)][keep], ref[keep],
                           rtol=1e-6, atol=0)
        # x is the wavefield: H x = b - r
        xr = spla.gmres(HB, b, rtol=1e-15, restart=8, maxiter=3)[0]
        assert np.linalg.norm(res.x - B @ xr) / np.linalg.norm(B @ xr) < 1e-7


def test_finite_termination_matches_lu():
    m = wl.smooth_slowness_2d(7, 9, 10.0, 1)
    f = wl.random_complex((7, 9), 2)
    omega = 2 * np.pi * 20
    res = solver.solve(m, omega, 0.01, 10.0, f, tol=1e-14, restart=63, maxiter=63,
                       precond="none")
    u = direct.solve_direct(m, omega, 0.01, 10.0, f)
    assert res.status == gm.OK
    assert np.linalg.norm(res.x - u) / np.linalg.norm(u) < 1e-10


@pytest.mark.parametrize("shape", [(200,), (13, 17)])
def test_one_iteration_when_preconditioner_is_exact_helmholtz(shape):
    """beta = (1, alpha) makes M = H; with an exact M^{-1} GMRES stops after one step."""
    m = (1.0 / wl.layered_velocity_1d(shape[0], 5.0) if len(shape) == 1
         else wl.smooth_slowness_2d(*shape, 10.0, 3))
    res = solver.solve(m, 2 * np.pi * 10, 0.01, 5.0, wl.random_complex(shape, 1),
                       beta=(1.0, 0.01), tol=1e-10, restart=10, precond="exact")
    assert res.iterations == 1 and res.status == gm.OK


def test_arnoldi_relation_and_orthonormality():
    w = wl.random_field_2d(65, 33, 10.0, seed=2, freq_hz=6.0, src=(32, 5))
    res = solver.solve(w.slowness, w.omega, w.alpha, w.h, w.source, tol=1e-12, restart=12,
                       maxiter=12, keep_basis=True)
    cyc = res.last_cycle
    V, Z, Hb, k = cyc["V"], cyc["Z"], cyc["Hbar"], cyc["k"]
    assert k == 12
    H = op.helmholtz(w.slowness, w.omega, w.alpha, w.h)
    SZ = np.stack([H @ z for z in Z], axis=1)
    VH = V.T @ Hb
    assert np.linalg.norm(SZ - VH) / np.linalg.norm(SZ) < 1e-12
    # modified Gram-Schmidt loses orthogonality in proportion to the condition
    # of the Krylov basis; a loose bound still catches a wrong projection
    assert np.abs(V.conj() @ V.T - np.eye(k + 1)).max() < 1e-6


def test_history_monotone_within_cycle_and_status():
    w = wl.layered_1d(301, 5.0, 10.0)
    res = solver.solve(w.slowness, w.omega, w.alpha, w.h, w.source, tol=1e-9, restart=7,
                       maxiter=400)
    h = np.array(res.history)
    assert res.status == gm.OK and res.true_rel_res <= 1e-9
    assert len(h) == res.iterations + 1 and h[0] == 1.0
    for c in range(0, len(h) - 1, 7):
        seg = h[c + 1: c + 8]
        assert np.all(np.diff(seg) <= 1e-15)
    res1 = solver.solve(w.slowness, w.omega, w.alpha, w.h, w.source, tol=1e-9, restart=7,
                        maxiter=1)
    assert res1.status == gm.NOT_CONVERGED and res1.iterations == 1 and len(res1.history) == 2


def test_zero_rhs():
    w = wl.layered_1d(51, src=10)
    res = solver.solve(w.slowness, w.omega, w.alpha, w.h, np.zeros(51, complex))
    assert res.iterations == 0 and res.status == gm.OK and not res.x.any()


# --------------------------------------------------------------------------
# the paper's qualitative claims (Section "Example")
# --------------------------------------------------------------------------
def test_layered_1d_preconditioned_vs_unpreconditioned():
    """Fig. 3-4: unpreconditioned GMRES converges slowly and does not model the
    data; preconditioned GMRES agrees with LU."""
    w = wl.layered_1d_well()
    pre = solver.solve(w.slowness, w.omega, w.alpha, w.h, w.source, beta=w.beta, tol=1e-6,
                       restart=50)
    raw = solver.solve(w.slowness, w.omega, w.alpha, w.h, w.source, tol=1e-6, restart=50,
                       maxiter=500, precond="none")
    u = direct.solve_direct(w.slowness, w.omega, w.alpha, w.h, w.source)
    assert pre.status == gm.OK and pre.iterations < 80
    assert raw.status == gm.NOT_CONVERGED and raw.true_rel_res > 1e-3
    err_pre = np.linalg.norm(pre.x - u) / np.linalg.norm(u)
    err_raw = np.linalg.norm(raw.x - u) / np.linalg.norm(u)
    assert err_pre < 1e-4 and err_raw > 0.1
    tight = solver.solve(w.slowness, w.omega, w.alpha, w.h, w.source, beta=w.beta, tol=1e-11,
                         restart=50)
    assert np.linalg.norm(tight.x - u) / np.linalg.norm(u) < 1e-6


def test_spectrum_claims_fig2():
    """Fig. 2 (1D model, 30 Hz, beta1 = beta2 = 1): H has eigenvalues at and left of
    the origin; M^{-1} H lies on the disc of centre (1+alpha)/2, radius
    (1-alpha)/2 and so has positive real parts."""
    n = 401
    m = 1.0 / wl.layered_velocity_1d(n, 12.5)
    omega, alpha = 2 * np.pi * 30, 0.01
    lam = spectrum.helmholtz_eigenvalues(m, omega, alpha, 12.5)
    mu = spectrum.preconditioned_eigenvalues(m, omega, alpha, 1.0, 1.0, 12.5)
    assert (lam.real < 0).sum() > 10
    c, r = spectrum.disc(alpha, 1.0)
    assert np.all(np.abs(mu - c) <= r * (1 + 1e-9))
    assert mu.real.min() > 0


@pytest.mark.parametrize("beta2", [0.5, 1.0])
def test_disc_bound_2d(beta2):
    m = wl.smooth_slowness_2d(9, 11, 10.0, 8)
    alpha = 0.01
    mu = spectrum.preconditioned_eigenvalues(m, 2 * np.pi * 25, alpha, 1.0, beta2, 10.0)
    c, r = spectrum.disc(alpha, beta2)
    assert np.all(np.abs(mu - c) <= r * (1 + 1e-9))


def test_iterations_mesh_independent_and_rise_with_frequency():
    """Introduction: with the preconditioner the iteration count does not grow
    with mesh refinement but does grow with the wavenumber."""
    its_h = []
    for n, h in ((501, 10.0), (1001, 5.0), (2001, 2.5)):
        w = wl.layered_1d(n, h, 10.0, src=int(round(500 / h)))
        its_h.append(solver.solve(w.slowness, w.omega, w.alpha, w.h, w.source,
                                  tol=1e-6, restart=200).iterations)
    assert max(its_h) - min(its_h) <= 0.15 * max(its_h), its_h
    its_f = []
    for f in (5.0, 10.0, 20.0):
        w = wl.layered_1d(2001, 2.5, f, src=200)
        its_f.append(solver.solve(w.slowness, w.omega, w.alpha, w.h, w.source,
                                  tol=1e-6, restart=200).iterations)
    assert its_f[0] < its_f[1] < its_f[2], its_f
