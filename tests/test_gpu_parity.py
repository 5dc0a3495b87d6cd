"""GPU parity: every step of the HIP path against the CPU FP64 oracle, through
the C ABI (ctypes binding), on the same seeded inputs.

Tolerances (FP64 throughout; the two sides differ only in rounding order):
* stencil / Galerkin operators:  max |y - y_ref| <= 1e-13 max |y_ref|
* tridiagonal solve / V-cycle:   ||z - z_ref|| <= 1e-10 ||z_ref||
* full solves: same iteration count (+-1), residual history within 1e-6
  relative while above 1e-12, wavefield within 1e-6 of the oracle's
  iterate (the spec bar) and true residual <= tol.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import workloads as wl                                         # noqa: E402
from oracle import operator as op, multigrid as mg, solver, direct, gmres as ogm  # noqa: E402


@pytest.fixture(scope="module")
def hh():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1712_08740_amd.hh as hh
    return hh


DEV = "cuda"


def _t(a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _np(t):
    return t.detach().cpu().numpy()


def _problem(hh, m, omega, alpha, h, beta=(1.0, 0.5)):
    return hh.Problem(_t(np.asarray(m, dtype=np.float64)), omega, alpha, h, beta=beta)


CASES_1D = [(1001, 5.0, 10.0), (37, 5.0, 10.0), (3, 5.0, 10.0), (1024, 5.0, 25.0)]
CASES_2D = [((201, 401), 10.0, 10.0), ((201, 401), 10.0, 15.0), ((13, 70), 10.0, 12.0),
            ((3, 3), 10.0, 10.0), ((65, 33), 10.0, 4.0), ((17, 9), 10.0, 2.0),
            ((129, 129), 10.0, 30.0)]


def _model(shape, h, seed=0):
    if len(shape) == 1:
        return 1.0 / wl.layered_velocity_1d(shape[0], h)
    if shape == (201, 401):
        return wl.grf_401x201().slowness
    return wl.smooth_slowness_2d(*shape, h, seed)


# ---------------------------------------------------------------------------
# operator apply (matrix-free stencil)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", CASES_1D + CASES_2D, ids=str)
def test_apply_operator(hh, case):
    shape, h, freq = (case[0],) if isinstance(case[0], int) else case[0], case[1], case[2]
    m = _model(shape, h)
    omega, alpha, beta = 2 * np.pi * freq, 0.01, (1.0, 0.5)
    P = _problem(hh, m, omega, alpha, h, beta)
    x = wl.random_complex(shape, 11)
    for which, A in (("H", op.helmholtz(m, omega, alpha, h)),
                     ("M", op.shifted_laplace(m, omega, *beta, h))):
        y = _np(P.apply_operator(_t(x), which))
        ref = (A @ x.ravel()).reshape(shape)
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max(), which


# ---------------------------------------------------------------------------
# multigrid hierarchy: level shapes and Galerkin operators
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", [c for c in CASES_2D if c[0] != (3, 3)], ids=str)
def test_level_operators_match_galerkin(hh, case):
    shape, h, freq = case
    m = _model(shape, h)
    omega = 2 * np.pi * freq
    P = _problem(hh, m, omega, 0.01, h)
    V = mg.VCycle(m, omega, 1.0, 0.5, h)
    assert P.num_levels == len(V.levels)
    for l, lev in enumerate(V.levels):
        (nz, nx), (hz, hx) = P.level_info(l)
        assert (nz, nx) == lev.shape
        assert (hz, hx) == lev.spacing
        x = wl.random_complex(lev.shape, 20 + l)
        y = _np(P.apply_level_operator(l, _t(x)))
        ref = (lev.M @ x.ravel()).reshape(lev.shape)
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max(), l


# ---------------------------------------------------------------------------
# preconditioner: exact tridiagonal solve (1D) and V-cycle (2D)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", CASES_1D, ids=str)
def test_pcr_matches_direct_solve(hh, case):
    n, h, freq = case
    m = _model((n,), h)
    omega = 2 * np.pi * freq
    P = _problem(hh, m, omega, 0.01, h)
    v = wl.random_complex((n,), 5)
    z = _np(P.apply_precond(_t(v)))
    ref = direct.solve_matrix(op.shifted_laplace(m, omega, 1.0, 0.5, h), v)
    assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)
    # and the residual of the solved system
    Mz = op.shifted_laplace(m, omega, 1.0, 0.5, h) @ z
    assert np.linalg.norm(Mz - v) <= 1e-10 * np.linalg.norm(v)


@pytest.mark.parametrize("case", CASES_2D, ids=str)
def test_vcycle_matches_oracle(hh, case):
    shape, h, freq = case
    m = _model(shape, h)
    omega = 2 * np.pi * freq
    P = _problem(hh, m, omega, 0.01, h)
    V = mg.VCycle(m, omega, 1.0, 0.5, h)
    for seed in (1, 2):
        v = wl.random_complex(shape, seed)
        z = _np(P.apply_precond(_t(v)))
        ref = V(v.ravel()).reshape(shape)
        assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)


def test_set_shift_rebuilds_hierarchy(hh):
    shape, h, freq = (65, 33), 10.0, 4.0
    m = _model(shape, h)
    omega = 2 * np.pi * freq
    P = _problem(hh, m, omega, 0.01, h)
    for beta in ((1.0, 1.0), (0.5, 0.25), (1.0, 0.5)):
        P.set_shift(*beta)
        V = mg.VCycle(m, omega, *beta, h)
        v = wl.random_complex(shape, 3)
        z = _np(P.apply_precond(_t(v)))
        ref = V(v.ravel()).reshape(shape)
        assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref), beta


# ---------------------------------------------------------------------------
# Arnoldi orthogonalisation (CGS2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,k", [(80601, 31), (1001, 51), (5000, 1), (257, 7)])
def test_orthogonalize(hh, n, k):
    rng = np.random.default_rng(n + k)
    A = rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))
    Q, _ = np.linalg.qr(A)
    V = np.ascontiguousarray(Q.T)
    w = wl.random_complex((n,), 9) + V.T @ (rng.standard_normal(k) * 3)
    wt = _t(w.copy())
    hvals, nrm = hh.orthogonalize(_t(V), wt)
    ref_h = V.conj() @ w
    w_out = _np(wt)
    ref_w = w - V.T @ ref_h
    assert np.abs(hvals - ref_h).max() <= 1e-12 * np.abs(ref_h).max()
    assert np.linalg.norm(w_out - ref_w) <= 1e-12 * np.linalg.norm(w)
    assert abs(nrm - np.linalg.norm(ref_w)) <= 1e-12 * np.linalg.norm(ref_w)
    assert np.abs(V.conj() @ w_out).max() <= 1e-13 * np.linalg.norm(w_out)


# ---------------------------------------------------------------------------
# full solves
# ---------------------------------------------------------------------------
def _check_solve(res, ref, tol, u_tol=1e-6):
    assert res.status == hh_ok()
    assert abs(res.iterations - ref.iterations) <= 1
    assert res.true_rel_res <= tol
    g = res.history
    r = np.asarray(ref.history)
    n = min(len(g), len(r))
    keep = r[:n] > 1e-12
    assert np.all(np.abs(g[:n][keep] - r[:n][keep]) <= 1e-6 * r[:n][keep])
    u = _np(res.u)
    assert np.linalg.norm(u - ref.x) <= u_tol * np.linalg.norm(ref.x)


def hh_ok():
    return 0


def test_solve_layered_1d_well(hh):
    w = wl.layered_1d_well()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h, w.beta)
    res = P.solve(_t(w.source), tol=w.tol, restart=w.restart)
    ref = solver.solve(w.slowness, w.omega, w.alpha, w.h, w.source, beta=w.beta, tol=w.tol,
                       restart=w.restart)
    assert ref.iterations == 49
    _check_solve(res, ref, w.tol)
    # against LU: tolerance scaled so the error meets 1e-6 (error ~ 18x residual here)
    res2 = P.solve(_t(w.source), tol=1e-10, restart=w.restart)
    u_lu = direct.solve_direct(w.slowness, w.omega, w.alpha, w.h, w.source)
    assert np.linalg.norm(_np(res2.u) - u_lu) <= 1e-6 * np.linalg.norm(u_lu)


def test_solve_grf_401x201(hh):
    w = wl.grf_401x201()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h, w.beta)
    res = P.solve(_t(w.source), tol=w.tol, restart=w.restart)
    ref = solver.solve(w.slowness, w.omega, w.alpha, w.h, w.source, beta=w.beta, tol=w.tol,
                       restart=w.restart)
    _check_solve(res, ref, w.tol)
    res2 = P.solve(_t(w.source), tol=1e-9, restart=w.restart)
    u_lu = direct.solve_direct(w.slowness, w.omega, w.alpha, w.h, w.source)
    assert np.linalg.norm(_np(res2.u) - u_lu) <= 1e-6 * np.linalg.norm(u_lu)
    assert res2.true_rel_res <= 1e-9


@pytest.mark.parametrize("shape,freq,restart", [((3, 3), 10.0, 5), ((5, 7), 10.0, 3),
                                                ((17, 9), 20.0, 4), ((13, 70), 12.0, 10),
                                                ((65, 33), 6.0, 30), ((3,), 10.0, 2),
                                                ((37,), 30.0, 5)], ids=str)
def test_solve_small_and_ragged(hh, shape, freq, restart):
    h = 10.0
    m = _model(shape, h, seed=4)
    omega = 2 * np.pi * freq
    f = wl.random_complex(shape, 8)
    P = _problem(hh, m, omega, 0.01, h)
    res = P.solve(_t(f), tol=1e-8, restart=restart, max_iters=500)
    ref = solver.solve(m, omega, 0.01, h, f, tol=1e-8, restart=restart, maxiter=500)
    _check_solve(res, ref, 1e-8)


def test_restart_one_matches_oracle(hh):
    """GMRES(1): every cycle is one Arnoldi step closed by the end-of-cycle
    projections (no step hosts a Givens update), so status, iteration count and
    residual history must follow the oracle step by step."""
    m = _model((37,), 10.0, seed=4)
    omega = 2 * np.pi * 5.0
    f = wl.random_complex((37,), 8)
    P = _problem(hh, m, omega, 0.01, 10.0)
    res = P.solve(_t(f), tol=1e-8, restart=1, max_iters=40)
    ref = solver.solve(m, omega, 0.01, 10.0, f, tol=1e-8, restart=1, maxiter=40)
    assert res.status == ref.status and res.iterations == ref.iterations
    n = min(len(res.history), len(ref.history))
    r = np.asarray(ref.history[:n])
    assert np.all(np.abs(res.history[:n] - r) <= 1e-6 * r)


def test_unpreconditioned_matches_oracle(hh):
    w = wl.layered_1d(301, 5.0, 10.0, src=50)
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    res = P.solve(_t(w.source), tol=1e-6, restart=20, max_iters=300, no_precond=True)
    ref = solver.solve(w.slowness, w.omega, w.alpha, w.h, w.source, tol=1e-6, restart=20,
                       maxiter=300, precond="none")
    assert res.status == ref.status
    assert res.iterations == ref.iterations
    n = min(len(res.history), len(ref.history))
    r = np.asarray(ref.history[:n])
    assert np.all(np.abs(res.history[:n] - r) <= 1e-6 * r)


def test_long_cycles_generic_basis_paths(hh):
    """Restart 80 without preconditioner on a 2D grid: the fused apply and the
    basis pass run their generic paths (more than 48 basis vectors, chunks of 8),
    the last column of a full cycle gets its own projections, and the cycle-end
    substitution runs its multi-wavefront form (restart > 32). Against the
    oracle's GMRES with the same parameters; a 3-source batch of the same runs
    the same kernels per source (no coarsest product) and equals its solves alone
    to the bit."""
    shape, h, freq = (17, 33), 10.0, 3.0
    m = _model(shape, h, seed=4)
    omega = 2 * np.pi * freq
    P = _problem(hh, m, omega, 0.01, h)
    f = np.zeros(shape, complex)
    f[8, 16] = 1.0
    kw = dict(tol=1e-6, restart=80, max_iters=1000, no_precond=True)
    res = P.solve(_t(f), **kw)
    ref = solver.solve(m, omega, 0.01, h, f, tol=1e-6, restart=80, maxiter=1000,
                       precond="none")
    print(f"restart 80 without preconditioner: {res.iterations} iterations "
          f"(oracle {ref.iterations})")
    assert res.iterations > 80                  # at least one full cycle
    assert res.status == ref.status == 0
    assert abs(res.iterations - ref.iterations) <= 1
    assert res.true_rel_res <= 1e-6
    n = min(80, len(res.history), len(ref.history))    # the first cycle step by step
    r = np.asarray(ref.history[:n])
    assert np.all(np.abs(res.history[:n] - r) <= 1e-6 * r)
    u = _np(res.u)
    assert np.linalg.norm(u - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
    F = _batch_sources(shape, [(8, 16), (0, 0), (16, 32)])
    _assert_batch_equals_single(P, F, exact=True, **kw)


def test_restart_at_its_maximum(hh):
    """restart = 1024 (the largest accepted): the basis and least-squares storage
    take their largest layout; unpreconditioned on a 2D grid the solve ends
    inside the one cycle, as the oracle's full GMRES does."""
    shape, h, freq = (17, 33), 10.0, 3.0
    m = _model(shape, h, seed=4)
    omega = 2 * np.pi * freq
    P = _problem(hh, m, omega, 0.01, h)
    f = np.zeros(shape, complex)
    f[8, 16] = 1.0
    res = P.solve(_t(f), tol=1e-6, restart=1024, max_iters=1000, no_precond=True)
    ref = solver.solve(m, omega, 0.01, h, f, tol=1e-6, restart=1024, maxiter=1000,
                       precond="none")
    assert res.status == ref.status == 0
    assert abs(res.iterations - ref.iterations) <= 1
    u = _np(res.u)
    assert np.linalg.norm(u - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


def test_batch_at_its_maximum_size(hh):
    """HH_MAX_BATCH sources of one small problem in one batch (32 groups of the
    batched coarsest product, the largest source grid dimension): every source
    converges and sampled sources equal their solves alone to rounding."""
    shape, h, freq = (9, 17), 10.0, 5.0
    m = _model(shape, h, seed=6)
    P = _problem(hh, m, 2 * np.pi * freq, 0.01, h)
    assert P.num_levels >= 3
    nrhs = hh.HH_MAX_BATCH
    F = np.stack([wl.random_complex(shape, 1000 + i) for i in range(nrhs)])
    kw = dict(tol=1e-8, restart=10)
    res = P.solve_batch(_t(F), **kw)
    assert res.overall == 0 and np.all(res.status == 0)
    U = _np(res.u)
    for i in (0, 1, 31, 32, 511, 640, 1022, 1023):
        one = P.solve(_t(F[i]), **kw)
        assert abs(int(res.iterations[i]) - one.iterations) <= 1, i
        bound = BATCH_REL if res.iterations[i] == one.iterations else 1e-6
        assert np.linalg.norm(U[i] - _np(one.u)) <= bound * np.linalg.norm(_np(one.u)), i


def test_zero_source_and_budget(hh):
    w = wl.layered_1d(101, 5.0, 10.0, src=10)
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    res = P.solve(_t(np.zeros(101, complex)), tol=1e-6, restart=10)
    assert res.status == 0 and res.iterations == 0 and not _np(res.u).any()
    assert list(res.history) == [1.0]
    res = P.solve(_t(w.source), tol=1e-6, restart=10, max_iters=1)
    assert res.status == 1 and res.iterations == 1 and len(res.history) == 2


def test_invalid_inputs(hh):
    m = _model((9, 11), 10.0)
    bad = m.copy()
    bad[3, 4] = np.nan
    with pytest.raises(hh.HHError) as e:
        _problem(hh, bad, 60.0, 0.01, 10.0)
    assert e.value.status == hh.HH_EINVAL
    bad[3, 4] = -1.0
    with pytest.raises(hh.HHError):
        _problem(hh, bad, 60.0, 0.01, 10.0)
    P = _problem(hh, m, 60.0, 0.01, 10.0)
    f = _t(wl.random_complex((9, 11), 1))
    for kw in (dict(tol=0.0), dict(tol=1.5), dict(restart=0), dict(max_iters=0)):
        args = dict(tol=1e-6, restart=5, max_iters=10)
        args.update(kw)
        with pytest.raises(hh.HHError) as e:
            P.solve(f, **args)
        assert e.value.status == hh.HH_EINVAL
    fbad = wl.random_complex((9, 11), 1)
    fbad[2, 2] = np.inf
    with pytest.raises(hh.HHError) as e:
        P.solve(_t(fbad), tol=1e-6, restart=5)
    assert e.value.status == hh.HH_ENUMERIC


def test_solve_grf_401x201_15hz_under_resolved_level(hh):
    """15 Hz: the hierarchy continues past two nodes per wavelength (51 x 101 has
    more than HH_MAX_COARSE nodes) and smooths that level with weight 0.5."""
    w = wl.random_field_2d(401, 201, 10.0, seed=2, freq_hz=15.0, src=(200, 5))
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h, w.beta)
    assert P.num_levels == 4 and P.level_info(3)[0] == (26, 51)
    res = P.solve(_t(w.source), tol=w.tol, restart=w.restart)
    ref = solver.solve(w.slowness, w.omega, w.alpha, w.h, w.source, beta=w.beta, tol=w.tol,
                       restart=w.restart)
    _check_solve(res, ref, w.tol)


def test_solve_is_bitwise_reproducible(hh):
    w = wl.grf_401x201()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    a = P.solve(_t(w.source), tol=w.tol, restart=w.restart)
    ua = _np(a.u).copy()
    b = P.solve(_t(w.source), tol=w.tol, restart=w.restart)
    assert np.array_equal(ua, _np(b.u))
    assert np.array_equal(a.history, b.history)


def test_restart_beyond_iteration_count_gives_same_bits(hh):
    """A restart length above the iteration count changes nothing but the
    storage of the least-squares factor: a solve that finishes inside one cycle
    gives the same bits for restart 40 and 600."""
    w = wl.grf_401x201()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    a = P.solve(_t(w.source), tol=w.tol, restart=40)
    b = P.solve(_t(w.source), tol=w.tol, restart=600)
    assert a.iterations == b.iterations
    assert np.array_equal(_np(a.u), _np(b.u))
    assert np.array_equal(a.history, b.history)


def _steps_per_cycle(iterations, restart):
    """Arnoldi steps taken per restart cycle: a full cycle takes restart steps
    (its last column is closed after them); a cycle that stops at column c
    learns it one step later, after c + 2 steps."""
    steps, left = [], iterations
    while left > restart:
        steps.append(restart)
        left -= restart
    steps.append(restart if left == restart else left + 1)
    return steps


def test_kernel_timer_counts_working_launches(hh):
    """The dispatch-stamped timer counts one launch per Arnoldi step that did work
    (steps enqueued ahead and skipped on the device are not counted) and sums the
    byte model (j + 4) * 16 B per node of the second Arnoldi pass at step j."""
    w = wl.grf_401x201()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    N = w.slowness.size
    P.kernel_timer_start("axpy_dot")
    res = P.solve(_t(w.source), tol=w.tol, restart=w.restart)
    launches, ms, nbytes = P.kernel_timer_read()
    steps = _steps_per_cycle(res.iterations, w.restart)
    assert launches == sum(steps)
    assert nbytes == pytest.approx(sum((j + 4) * 16.0 * N for c in steps for j in range(c)),
                                   rel=1e-12)
    assert 0 < ms < 1e3
    P.kernel_timer_start("none")


@pytest.mark.gpu
def test_kernel_timer_classes_cover_the_step(hh):
    """Every kernel class of a 2D multigrid step is timed with one launch per
    working step (per level for the coarse legs); a full cycle adds the
    projections of its last vector (axpy_norm class), one reduction and the
    Givens step that closes it; the byte model of the fine down leg is 56 B
    per fine node + 16 B per coarse node."""
    w = wl.grf_401x201()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    N = w.slowness.size
    nl = P.num_levels
    shapes = [P.level_shape(l) for l in range(nl)]
    res = P.solve(_t(w.source), tol=w.tol, restart=w.restart)
    it = res.iterations
    assert it == w.restart + 6
    steps = sum(_steps_per_cycle(it, w.restart))
    full = it // w.restart
    expect = {"apply_dot": steps, "axpy_dot": steps, "reduce": steps + full,
              "vc_down": steps, "vc_up": steps, "gemv": steps,
              "vc_down_coarse": (nl - 2) * steps, "vc_up_coarse": (nl - 2) * steps,
              "axpy_norm": full, "givens": full, "pcr": 0}
    for k, n in expect.items():
        P.kernel_timer_start(k)
        r = P.solve(_t(w.source), tol=w.tol, restart=w.restart)
        launches, ms, nbytes = P.kernel_timer_read()
        assert r.iterations == it
        assert launches == n, k
        assert (ms > 0) == (n > 0), k
        if k == "vc_down":
            n1 = shapes[1][0] * shapes[1][1]
            assert nbytes == pytest.approx(steps * (56.0 * N + 16.0 * n1), rel=1e-12)
    P.kernel_timer_start("none")


# ---------------------------------------------------------------------------
# single-precision preconditioner inside the FP64 flexible GMRES
# ---------------------------------------------------------------------------
# The complex64 cycle rounds its data (m^2, omega_J/diag, Galerkin planes,
# coarsest inverse) and its arithmetic to 24-bit mantissas: its output differs
# from the FP64 cycle by about eps32 = 6e-8 times the cycle's amplification of
# data perturbations. Measured on the grids below: 7.5e-8 (3 x 3) to 5.9e-7
# (129 x 129 at 30 Hz), i.e. amplification <= 10; the bound allows 80.
F32_CYCLE_TOL = 5e-6


@pytest.mark.parametrize("case", CASES_2D, ids=str)
def test_vcycle_f32_matches_oracle(hh, case):
    shape, h, freq = case
    m = _model(shape, h)
    omega = 2 * np.pi * freq
    P = _problem(hh, m, omega, 0.01, h)
    V = mg.VCycle(m, omega, 1.0, 0.5, h)
    for seed in (1, 2):
        v = wl.random_complex(shape, seed)
        z = _np(P.apply_precond(_t(v), f32=True))
        assert z.dtype == np.complex64
        ref = V(v.ravel()).reshape(shape)
        err = np.linalg.norm(z.astype(np.complex128) - ref) / np.linalg.norm(ref)
        print(f"f32 cycle {shape} {freq} Hz seed {seed}: rel err {err:.2e}")
        assert err <= F32_CYCLE_TOL


@pytest.mark.parametrize("n", [1001, 37])
def test_pcr_f32_matches_direct_solve(hh, n):
    h, freq = 5.0, 10.0
    m = _model((n,), h)
    omega = 2 * np.pi * freq
    P = _problem(hh, m, omega, 0.01, h)
    v = wl.random_complex((n,), 5)
    z = _np(P.apply_precond(_t(v), f32=True)).astype(np.complex128)
    ref = direct.solve_matrix(op.shifted_laplace(m, omega, 1.0, 0.5, h), v)
    assert np.linalg.norm(z - ref) <= F32_CYCLE_TOL * np.linalg.norm(ref)


def test_solve_f32_precond_401x201(hh):
    """Mixed precision at the 401 x 201 workload: the tolerance is met in full
    precision (recomputed residual), with about the FP64 iteration count; at a
    tolerance scaled as for the FP64 path the wavefield matches LU to 1e-6."""
    w = wl.grf_401x201()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    r64 = P.solve(_t(w.source), tol=w.tol, restart=w.restart)
    r32 = P.solve(_t(w.source), tol=w.tol, restart=w.restart, precond_f32=True)
    assert r32.status == 0 and r32.true_rel_res <= w.tol
    assert abs(r32.iterations - r64.iterations) <= 2
    H = op.helmholtz(w.slowness, w.omega, w.alpha, w.h)
    b = op.weighted_rhs(w.source).ravel()
    u = _np(r32.u).ravel()
    assert np.linalg.norm(b - H @ u) <= w.tol * np.linalg.norm(b)
    lu = direct.solve_direct(w.slowness, w.omega, w.alpha, w.h, w.source).ravel()
    tight = P.solve(_t(w.source), tol=1e-9, restart=w.restart, precond_f32=True)
    ut = _np(tight.u).ravel()
    assert np.linalg.norm(ut - lu) <= 1e-6 * np.linalg.norm(lu)


def test_solve_f32_precond_1201x401_15hz(hh):
    """The mixed-precision configuration: 1201 x 401, 15 Hz, FGMRES(40), tol 1e-8.
    The recomputed FP64 residual (oracle operator on the CPU) meets 1e-8."""
    w = wl.grf_1201x401()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    r32 = P.solve(_t(w.source), tol=w.tol, restart=w.restart, precond_f32=True)
    print(f"1201x401 15 Hz mixed: {r32.iterations} iterations, rel res {r32.true_rel_res:.3e}")
    assert r32.status == 0 and r32.true_rel_res <= w.tol
    H = op.helmholtz(w.slowness, w.omega, w.alpha, w.h)
    b = op.weighted_rhs(w.source).ravel()
    u = _np(r32.u).ravel()
    rel = np.linalg.norm(b - H @ u) / np.linalg.norm(b)
    assert rel <= w.tol * (1 + 1e-6)
    r64 = P.solve(_t(w.source), tol=w.tol, restart=w.restart)
    print(f"1201x401 15 Hz FP64: {r64.iterations} iterations")
    assert abs(r32.iterations - r64.iterations) <= max(2, r64.iterations // 20)
    assert np.linalg.norm(u - _np(r64.u).ravel()) <= 1e-6 * np.linalg.norm(u)


@pytest.mark.gpu
def test_stagnating_cycles_keep_the_basis_in_range(hh):
    """Regression: the Arnoldi step preconditions the stored vector before it
    is normalised, so that vector must be rescaled every step. On a grid whose
    hierarchy stalls FGMRES (1601 x 601 at 10 Hz with the 4096-node dense limit:
    the residual stays near 0.11), unscaled vectors grow by the product of the
    subdiagonal entries and overflowed complex64 within one 30-step cycle. Both
    precisions must stay finite and give the same residual history."""
    w = wl.random_field_2d(1601, 601, 10.0, seed=1001, freq_hz=10.0, src=(800, 5))
    P = hh.Problem(_t(w.slowness), w.omega, 0.01, 10.0, max_coarse=4096)
    r64 = P.solve(_t(w.source), tol=1e-6, restart=30, max_iters=90)
    r32 = P.solve(_t(w.source), tol=1e-6, restart=30, max_iters=90, precond_f32=True)
    P.close()
    for r in (r64, r32):
        assert r.status == hh.HH_NOT_CONVERGED and r.iterations == 90
        assert np.all(np.isfinite(r.history)) and 0.05 < r.true_rel_res < 0.5
    np.testing.assert_allclose(r32.history, r64.history, rtol=1e-3)


def test_f32_flag_validation(hh):
    w = wl.layered_1d_well()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    with pytest.raises(hh.HHError):
        P.solve(_t(w.source), tol=1e-6, restart=5, no_precond=True, precond_f32=True)
    r = P.solve(_t(w.source), tol=w.tol, restart=w.restart, precond_f32=True)
    assert r.status == 0 and r.true_rel_res <= w.tol


# ---------------------------------------------------------------------------
# several sources of one problem solved together (hh_solve_batch)
# ---------------------------------------------------------------------------
def _batch_sources(shape, positions):
    F = np.zeros((len(positions),) + tuple(shape), dtype=np.complex128)
    for i, pos in enumerate(positions):
        if pos is not None:
            F[(i,) + tuple(pos)] = 1.0
    return F


# A batch applies the coarsest inverse to all its sources as one GEMM, whose
# summation order differs from the single solve's matrix-vector product; every
# other operation is the same per source. The two iterations therefore differ
# by rounding (1e-16 per product, carried through at most a few hundred steps):
# same iteration count (a convergence test sitting on the tolerance may flip by
# one), and with equal counts the wavefields agree to 1e-10 (complex128
# preconditioner) or 1e-8 (complex64 preconditioner: its rounding differences
# are eps32 = 6e-8 per product instead of 1e-16; measured 2e-10 on 801 x 301);
# with counts one apart both have met the tolerance and agree to the 1e-6 bar.
BATCH_REL = 1e-10
BATCH_REL_F32 = 1e-8


def _assert_batch_equals_single(P, F, exact=False, **kw):
    """Every source of a batch gives its solve alone, to rounding (to the bit
    where no GEMM is involved: exact)."""
    res = P.solve_batch(_t(F), **kw)
    for i in range(F.shape[0]):
        one = P.solve(_t(F[i]), **kw)
        if exact:
            assert res.iterations[i] == one.iterations, i
            assert np.array_equal(_np(res.u[i]), _np(one.u)), i
        assert abs(int(res.iterations[i]) - one.iterations) <= 1, i
        assert res.status[i] == one.status, i
        u, u1 = _np(res.u[i]), _np(one.u)
        same = BATCH_REL_F32 if kw.get("precond_f32") else BATCH_REL
        bound = same if res.iterations[i] == one.iterations else 1e-6
        assert np.linalg.norm(u - u1) <= bound * max(np.linalg.norm(u1), 1e-300), i
    return res


def test_batch_equals_single_solves_401x201(hh):
    """Sources at different depths converge after different iteration counts
    (some restart, some do not); a zero source is done at once."""
    w = wl.grf_401x201()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    F = _batch_sources(w.shape, [(5, 200), (100, 37), None, (200, 400), (0, 0)])
    res = _assert_batch_equals_single(P, F, tol=w.tol, restart=w.restart)
    assert res.overall == 0 and np.all(res.status == 0)
    assert res.iterations[2] == 0
    assert len(set(res.iterations.tolist())) >= 3
    # one of them against the oracle
    ref = solver.solve(w.slowness, w.omega, w.alpha, w.h, F[1], beta=w.beta, tol=w.tol,
                       restart=w.restart)
    assert abs(res.iterations[1] - ref.iterations) <= 1
    assert np.linalg.norm(_np(res.u[1]) - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("kw", [dict(restart=7, tol=1e-8), dict(restart=12, tol=1e-7,
                                                               precond_f32=True),
                                dict(restart=20, tol=1e-6, no_precond=True, max_iters=400)],
                         ids=["f64_restarts", "f32", "no_precond"])
def test_batch_equals_single_small_grid(hh, kw):
    shape, h, freq = (33, 65), 10.0, 6.0
    m = _model(shape, h, seed=3)
    P = _problem(hh, m, 2 * np.pi * freq, 0.01, h)
    F = _batch_sources(shape, [(3, 10), (16, 32), (32, 64), (1, 1), (20, 5), (7, 50), (30, 3),
                               (12, 12), (25, 60)])
    res = _assert_batch_equals_single(P, F, **kw)
    H = op.helmholtz(m, 2 * np.pi * freq, 0.01, h)
    for i in range(F.shape[0]):
        b = op.weighted_rhs(F[i]).ravel()
        r = np.linalg.norm(b - H @ _np(res.u[i]).ravel()) / np.linalg.norm(b)
        if res.status[i] == 0:
            assert r <= kw["tol"] * (1 + 1e-6)


@pytest.mark.parametrize("kw", [dict(restart=10, tol=1e-8),
                                dict(restart=10, tol=1e-7, precond_f32=True)],
                         ids=["f64", "f32"])
@pytest.mark.parametrize("shape", [(45, 97), (49, 97)], ids=["nc156", "nc91"])
def test_batch_two_source_groups_ragged_coarsest(hh, kw, shape):
    """37 sources: the batched coarsest product runs a full group of 32 and a
    partial one of 5; the grid makes every level (and the coarsest size) ragged
    against the product's 16-entry steps and 128-row blocks; an even and an odd
    coarsest size (the complex64 product loads entry pairs only when rows are
    16-byte aligned)."""
    h, freq = 10.0, 5.0
    m = _model(shape, h, seed=8)
    P = _problem(hh, m, 2 * np.pi * freq, 0.01, h)
    nc = int(np.prod(P.level_info(P.num_levels - 1)[0]))
    assert P.num_levels >= 3 and nc % 16 != 0
    rng = np.random.default_rng(37)
    pos = [(int(rng.integers(0, shape[0])), int(rng.integers(0, shape[1]))) for _ in range(37)]
    F = _batch_sources(shape, pos)
    res = _assert_batch_equals_single(P, F, **kw)
    assert np.all(res.status == 0)


@pytest.mark.parametrize("f32", [False, True], ids=["f64", "f32"])
def test_batch_is_bitwise_reproducible(hh, f32):
    """The batched coarsest product (matrix cores, split over k) adds its terms
    and partial sums in a fixed order: two batched solves give the same bits."""
    w = wl.grf_401x201()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    F = _t(_batch_sources(w.shape, [(5, 200), (100, 37), (200, 400), (0, 0), (150, 300)]))
    a = P.solve_batch(F, tol=w.tol, restart=w.restart, precond_f32=f32)
    ua = _np(a.u).copy()
    b = P.solve_batch(F, tol=w.tol, restart=w.restart, precond_f32=f32)
    assert np.array_equal(a.iterations, b.iterations)
    assert np.array_equal(_np(b.u), ua)


@pytest.mark.parametrize("shape", [(1001,), (3, 3)], ids=str)
def test_batch_1d_and_single_level(hh, shape):
    if len(shape) == 1:
        w = wl.layered_1d_well()
        m, omega, h = w.slowness, w.omega, w.h
        pos = [(100,), (500,), (1000,), (0,)]
    else:
        m, omega, h = _model(shape, 10.0), 2 * np.pi * 10.0, 10.0
        pos = [(0, 0), (1, 1), (2, 1)]
    P = _problem(hh, m, omega, 0.01, h)
    F = _batch_sources(shape, pos)
    # exact 1D solve / fine grid = coarsest level: the batch runs the same
    # kernels per source (no GEMM), so the bits agree
    _assert_batch_equals_single(P, F, exact=True, tol=1e-8, restart=10)
    _assert_batch_equals_single(P, F, exact=True, tol=1e-8, restart=10, precond_f32=True)


BATCH_MAX_COARSE = 16384


def test_batch_801x301_32_sources_per_frequency(hh):
    """The batching configuration at full size: 801 x 301, 32 top-row sources at
    each of 5 / 7.5 / 10 / 12.5 Hz (one problem per frequency, 32 sources per
    batch, coarsest dense limit 16384). Every source meets 1e-6 on the residual
    recomputed in FP64 by the oracle's operator; two sources per frequency equal
    their solves alone."""
    slow, sources, freqs = wl.grf_801x301_sources()
    shape = slow.shape
    F = _batch_sources(shape, [(iz, ix) for ix, iz in sources])
    for fz in freqs:
        omega = 2 * np.pi * fz
        P = _problem(hh, slow, omega, 0.01, 10.0)
        P.set_max_coarse(BATCH_MAX_COARSE)
        res = P.solve_batch(_t(F), tol=1e-6, restart=30, precond_f32=True)
        print(f"801x301 {fz} Hz: iterations {res.iterations.min()}..{res.iterations.max()}")
        assert res.overall == 0 and np.all(res.status == 0)
        H = op.helmholtz(slow, omega, 0.01, 10.0)
        U = _np(res.u)
        for i in range(F.shape[0]):
            b = op.weighted_rhs(F[i]).ravel()
            assert np.linalg.norm(b - H @ U[i].ravel()) <= 1e-6 * (1 + 1e-6) * np.linalg.norm(b)
        for i in (0, 17):
            one = P.solve(_t(F[i]), tol=1e-6, restart=30, precond_f32=True)
            assert abs(one.iterations - int(res.iterations[i])) <= 1
            bound = BATCH_REL_F32 if one.iterations == res.iterations[i] else 1e-6
            assert np.linalg.norm(_np(one.u) - U[i]) <= bound * np.linalg.norm(U[i])
        del P, res
        torch.cuda.empty_cache()


def test_batch_argument_checks(hh):
    w = wl.layered_1d_well()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    F = _t(np.zeros((2, 1001), complex))
    with pytest.raises(ValueError):
        P.solve_batch(_t(np.zeros((2, 1000), complex)))
    with pytest.raises(hh.HHError):
        P.solve_batch(F, tol=2.0)
    with pytest.raises(hh.HHError):
        P.solve_batch(F, restart=0)
    small = torch.empty(16, dtype=torch.uint8, device=DEV)
    with pytest.raises(ValueError):
        P.solve_batch(F, workspace=small)
    res = P.solve_batch(F, tol=1e-6, restart=5)
    assert np.all(res.iterations == 0) and np.all(res.status == 0)
    assert float(torch.abs(res.u).max()) == 0.0


@pytest.mark.parametrize("fz", [12.5, 5.0])
def test_max_coarse_hierarchy_matches_oracle(hh, fz):
    """A larger dense limit: same levels as the oracle's rule with that limit,
    the cycle equals the oracle's, and the solve takes the oracle's iteration
    count (12.5 Hz on 801 x 301: 74 instead of 427 with the default limit)."""
    slow, sources, _ = wl.grf_801x301_sources()
    omega = 2 * np.pi * fz
    P = _problem(hh, slow, omega, 0.01, 10.0)
    P.set_max_coarse(BATCH_MAX_COARSE)
    V = mg.VCycle(slow, omega, 1.0, 0.5, 10.0, max_coarse=BATCH_MAX_COARSE)
    assert [P.level_shape(l) for l in range(P.num_levels)] == [l.shape for l in V.levels]
    v = wl.random_complex(slow.shape, 4)
    z = _np(P.apply_precond(_t(v)))
    ref = V(v.ravel()).reshape(slow.shape)
    assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)
    z32 = _np(P.apply_precond(_t(v), f32=True)).astype(np.complex128)
    assert np.linalg.norm(z32 - ref) <= F32_CYCLE_TOL * np.linalg.norm(ref)
    f = np.zeros(slow.shape, complex)
    f[0, sources[0][0]] = 1.0
    res = P.solve(_t(f), tol=1e-6, restart=30)
    H = op.helmholtz(slow, omega, 0.01, 10.0)
    b = op.weighted_rhs(f)
    ref = ogm.gmres(lambda x: H @ x, b, 1e-6, 30, 800, prec=V, flexible=True)
    ref.x = ref.x.reshape(slow.shape)
    print(f"801x301 {fz} Hz, dense limit {BATCH_MAX_COARSE}: GPU {res.iterations}, "
          f"oracle {ref.iterations}")
    _check_solve(res, ref, 1e-6)


def test_max_coarse_argument_checks(hh):
    w = wl.grf_401x201()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    for bad in (0, hh.HH_MAX_COARSE_LIMIT + 1):
        with pytest.raises(hh.HHError):
            P.set_max_coarse(bad)
    P.set_max_coarse(1000)            # coarsens further: 26 x 51 -> 26 x 26
    assert P.level_shape(P.num_levels - 1) == (26, 26)
    res = P.solve(_t(w.source), tol=w.tol, restart=w.restart)
    assert res.status == 0 and res.true_rel_res <= w.tol
    # 26 x 26 cannot be halved again: unsupported, and the previous hierarchy stays
    with pytest.raises(hh.HHError):
        P.set_max_coarse(100)
    assert P.level_shape(P.num_levels - 1) == (26, 26)
    res = P.solve(_t(w.source), tol=w.tol, restart=w.restart)
    assert res.status == 0 and res.true_rel_res <= w.tol
    P.set_max_coarse(hh.HH_MAX_COARSE)
    assert P.level_shape(P.num_levels - 1) == (26, 51)
    w1 = wl.layered_1d_well()
    P1 = _problem(hh, w1.slowness, w1.omega, w1.alpha, w1.h)
    with pytest.raises(hh.HHError):
        P1.set_max_coarse(8192)


# ---------------------------------------------------------------------------
# tile shapes of the multigrid legs and their autotuner
# ---------------------------------------------------------------------------
def test_every_tile_shape_gives_the_same_bits(hh):
    """Each leg's tile shape changes only how nodes are grouped into blocks:
    the preconditioner output is the same to the bit for every shape of every
    leg (complex128 and complex64 cycles), and for all levels changed at once."""
    w = wl.grf_401x201()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    nlegs = P.num_levels - 1
    assert nlegs >= 3
    v = _t(wl.random_complex(w.shape, 21))
    for f32 in (False, True):
        z0 = _np(P.apply_precond(v, f32=f32))
        for l in range(nlegs):
            for d in range(hh.HH_TILE_DOWN_COUNT):
                for u in range(hh.HH_TILE_UP_COUNT):
                    P.set_tiles(l, d, u)
                    assert np.array_equal(_np(P.apply_precond(v, f32=f32)), z0), (f32, l, d, u)
            P.set_tiles(l, -1, -1)
        for d, u in ((1, 1), (0, 2), (1, 0)):
            for l in range(nlegs):
                P.set_tiles(l, d, u)
            assert np.array_equal(_np(P.apply_precond(v, f32=f32)), z0), (f32, d, u)
        for l in range(nlegs):
            P.set_tiles(l, -1, -1)


@pytest.mark.parametrize("shape", [(9, 9), (5, 129), (13, 21), (33, 65), (65, 117)], ids=str)
def test_marching_down_leg_gives_the_tiled_bits(hh, shape):
    """The fine level's down leg marching along z (58-column strips, 8-row
    chunks) against the 4 x 4 tiles on grids smaller than one strip or chunk
    and ragged against both: the same bits, complex128 and complex64, and for a
    batch of sources."""
    h, freq = 10.0, 6.0
    m = _model(shape, h, seed=9)
    P = _problem(hh, m, 2 * np.pi * freq, 0.01, h)
    if P.num_levels < 2:
        pytest.skip("single-level hierarchy")
    v = _t(wl.random_complex(shape, 31))
    for f32 in (False, True):
        P.set_tiles(0, 0, -1)                       # 4 x 4 tiles
        z0 = _np(P.apply_precond(v, f32=f32))
        P.set_tiles(0, 2, -1)                       # marching along z
        assert np.array_equal(_np(P.apply_precond(v, f32=f32)), z0), f32
    F = _t(np.stack([wl.random_complex(shape, 40 + i) for i in range(3)]))
    P.set_tiles(0, 0, -1)
    a = P.solve_batch(F, tol=1e-8, restart=10, precond_f32=True)
    ua = _np(a.u).copy()
    P.set_tiles(0, 2, -1)
    b = P.solve_batch(F, tol=1e-8, restart=10, precond_f32=True)
    assert np.array_equal(a.iterations, b.iterations)
    assert np.array_equal(_np(b.u), ua)


def test_autotune_keeps_results_and_caches_choices(hh, tmp_path):
    """The tuner picks a valid shape per leg (or keeps the default); a solve with the tuned shapes
    gives the bits of the default ones; a second handle on the same hierarchy
    takes the choice from the cache file."""
    w = wl.grf_401x201()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    ref = P.solve(_t(w.source), tol=w.tol, restart=w.restart)
    u_ref = _np(ref.u).copy()
    cache = str(tmp_path / "tiles.json")
    tiles = P.autotune(cache=cache)
    assert len(tiles) == P.num_levels - 1
    for l, (d, u) in enumerate(tiles):
        assert -1 <= d < hh.HH_TILE_DOWN_COUNT and -1 <= u < hh.HH_TILE_UP_COUNT
        assert P.get_tiles(l) == (d, u)
    res = P.solve(_t(w.source), tol=w.tol, restart=w.restart)
    assert res.iterations == ref.iterations
    assert np.array_equal(_np(res.u), u_ref)
    key = hh.tile_cache_key([P.level_info(l)[0] for l in range(P.num_levels)], False, 1)
    assert hh.read_tile_cache(cache)[key] == [list(t) for t in tiles]
    Q = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    # a planted entry shows that the cache is read, not re-timed
    planted = [(1, 1)] * len(tiles)
    hh.write_tile_cache(cache, key, planted)
    assert Q.autotune(cache=cache) == planted
    assert all(Q.get_tiles(l) == (1, 1) for l in range(len(tiles)))
    # the complex64 cycle for batches of 4 is another entry
    tiles4 = Q.autotune(precond_f32=True, nrhs=4, cache=cache)
    assert len(hh.read_tile_cache(cache)) == 2 and len(tiles4) == len(tiles)


def test_autotuned_batch_gives_the_same_bits(hh):
    shape, h, freq = (65, 129), 10.0, 8.0
    m = wl.smooth_slowness_2d(*shape, h, 5)
    P = _problem(hh, m, 2 * np.pi * freq, 0.01, h)
    F = _t(_batch_sources(shape, [(3, 64), (32, 5), (60, 120)]))
    kw = dict(tol=1e-7, restart=9, precond_f32=True)
    a = P.solve_batch(F, **kw)
    ua = _np(a.u).copy()
    P.autotune(precond_f32=True, nrhs=3, reps=3)
    b = P.solve_batch(F, **kw)
    assert np.array_equal(b.iterations, a.iterations)
    assert np.array_equal(_np(b.u), ua)


def test_tile_argument_checks(hh):
    w = wl.grf_401x201()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    nl = P.num_levels
    for bad in ((nl - 1, 0, 0), (-1, 0, 0), (0, hh.HH_TILE_DOWN_COUNT, 0),
                (0, 0, hh.HH_TILE_UP_COUNT), (0, -2, 0)):
        with pytest.raises(hh.HHError):
            P.set_tiles(*bad)
    with pytest.raises(hh.HHError):
        P.get_tiles(nl - 1)
    ws = torch.empty(16, dtype=torch.uint8, device=DEV)
    with pytest.raises(hh.HHError):
        hh._check(hh._lib.hh_autotune(P._handle, 0, 1, hh._vp(ws.data_ptr()), 16, 10, None),
                  "hh_autotune")
    g = wl.layered_1d_well()
    Q = _problem(hh, g.slowness, g.omega, g.alpha, g.h)
    assert Q.autotune() == []
    with pytest.raises(hh.HHError):
        Q.get_tiles(0)


# ---------------------------------------------------------------------------
# initial guess: resuming a stopped solve (HH_INITIAL_GUESS)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("f32", [False, True], ids=["f64", "f32"])
def test_resume_at_a_cycle_boundary_gives_the_same_bits(hh, f32):
    """Restarted GMRES carries nothing across a restart but the iterate: a
    solve stopped by its budget at the end of a cycle and resumed from the
    returned u gives the uninterrupted solve's bits, the iterations adding up;
    the resumed history starts at the stopped solve's true residual."""
    w = wl.grf_401x201()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    f = _t(w.source)
    kw = dict(tol=w.tol, restart=10, precond_f32=f32)
    full = P.solve(f, max_iters=2000, **kw)
    assert full.status == hh.HH_OK and full.iterations > 20
    part = P.solve(f, max_iters=20, **kw)
    assert part.status == hh.HH_NOT_CONVERGED and part.iterations == 20
    rest = P.solve(f, max_iters=2000, x0=part.u.clone(), **kw)
    assert rest.status == hh.HH_OK
    assert rest.iterations + 20 == full.iterations
    assert np.array_equal(_np(rest.u), _np(full.u))
    assert rest.history[0] == pytest.approx(part.true_rel_res, rel=1e-12)
    assert rest.true_rel_res == full.true_rel_res


def test_initial_guess_edge_cases(hh):
    """From the converged solution no iteration is taken and u keeps its bits;
    a zero source returns u = 0 whatever the guess; from a guess stopped in the
    middle of a cycle the solve still meets the tolerance on the residual."""
    w = wl.grf_401x201()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    f = _t(w.source)
    done = P.solve(f, tol=w.tol, restart=w.restart)
    again = P.solve(f, tol=w.tol, restart=w.restart, x0=done.u.clone())
    assert again.status == hh.HH_OK and again.iterations == 0
    assert np.array_equal(_np(again.u), _np(done.u))
    assert again.history[0] == pytest.approx(done.true_rel_res, rel=1e-12)
    junk = _t(wl.random_complex(w.shape, 11))
    zero = P.solve(torch.zeros_like(f), tol=w.tol, restart=w.restart, x0=junk)
    assert zero.status == hh.HH_OK and zero.iterations == 0
    assert not torch.any(zero.u != 0)
    bad = done.u.clone()
    bad[3, 7] = complex(float("nan"), 0.0)
    with pytest.raises(hh.HHError) as e:       # a non-finite guess is a non-finite residual
        P.solve(f, tol=w.tol, restart=w.restart, x0=bad)
    assert e.value.status == hh.HH_ENUMERIC
    mid = P.solve(f, tol=w.tol, restart=w.restart, max_iters=13)
    assert mid.status == hh.HH_NOT_CONVERGED
    rest = P.solve(f, tol=w.tol, restart=w.restart, x0=mid.u.clone())
    assert rest.status == hh.HH_OK and rest.true_rel_res <= w.tol
    # the residual recomputed in FP64 by the oracle's operator
    H = op.helmholtz(w.slowness, w.omega, w.alpha, w.h)
    b = op.weighted_rhs(w.source).ravel()
    r = np.linalg.norm(b - H @ _np(rest.u).ravel())
    assert r <= w.tol * (1 + 1e-6) * np.linalg.norm(b)


def test_batch_resume_at_a_cycle_boundary(hh):
    """The batch resumes the same way, source by source: a source that had
    converged stays converged with no iteration, a zero source returns zero from
    a non-zero guess, and the rest give the uninterrupted batch's bits."""
    w = wl.grf_401x201()
    P = _problem(hh, w.slowness, w.omega, w.alpha, w.h)
    F = _t(_batch_sources(w.shape, [(5, 200), (100, 37), None, (200, 400)]))
    kw = dict(tol=w.tol, restart=10)
    full = P.solve_batch(F, max_iters=2000, **kw)
    assert full.overall == 0 and full.iterations[2] == 0
    part = P.solve_batch(F, max_iters=20, **kw)
    X0 = part.u.clone()
    X0[2] = _t(wl.random_complex(w.shape, 12))
    rest = P.solve_batch(F, max_iters=2000, X0=X0, **kw)
    assert rest.overall == 0 and np.all(rest.status == 0)
    assert not torch.any(rest.u[2] != 0) and rest.iterations[2] == 0
    for i in (0, 1, 3):
        if part.status[i] == hh.HH_OK:
            assert rest.iterations[i] == 0
            assert np.array_equal(_np(rest.u[i]), _np(part.u[i])), i
        else:
            assert part.iterations[i] == 20
            assert rest.iterations[i] + 20 == full.iterations[i], i
            assert np.array_equal(_np(rest.u[i]), _np(full.u[i])), i
