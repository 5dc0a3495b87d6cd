"""Admission logic of the request loop (CPU: the solve is replaced by a timed
stand-in, so only the scheduling is exercised) and, on the GPU, results of a
mixed stream against the same solves run alone."""
import threading
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1712_08740_amd import serve   # noqa: E402


class Probe:
    """Stand-in solve: holds its footprint for a while and records the peak
    memory and concurrency the server allowed."""

    def __init__(self, budget):
        self.budget = budget
        self.lock = threading.Lock()
        self.in_use = 0
        self.running = 0
        self.peak = 0
        self.peak_running = 0
        self.order = []

    def footprint(self, req):
        return int(req.slowness.size)          # a request's size stands for its bytes

    def solve(self, req, device, stream):
        fp = self.footprint(req)
        with self.lock:
            self.in_use += fp
            self.running += 1
            self.peak = max(self.peak, self.in_use)
            self.peak_running = max(self.peak_running, self.running)
            self.order.append(req.id)
            assert self.in_use <= self.budget
        time.sleep(0.02 + 0.00001 * fp)
        with self.lock:
            self.in_use -= fp
            self.running -= 1
        return serve.Result(id=req.id, u=np.zeros(1), iterations=1, true_rel_res=0.0, status=0,
                            footprint=0, t_arrival=0.0, t_admit=0.0, t_done=0.0)


def _req(i, size):
    return serve.Request(id=i, slowness=np.ones(size), h=1.0, freq_hz=1.0,
                         source=np.zeros(size, complex))


def test_admission_respects_budget_and_overlaps():
    budget = 1000
    pr = Probe(budget)
    srv = serve.Server(budget, workers=4, device=None, solve_fn=pr.solve,
                       footprint_fn=pr.footprint)
    sizes = [300, 300, 300, 900, 100, 100, 500, 200, 200, 50] * 3
    for i, sz in enumerate(sizes):
        srv.submit(_req(i, sz))
    res = srv.results(timeout=30)
    srv.close()
    assert sorted(res) == list(range(len(sizes)))
    assert pr.peak <= budget and srv.peak_in_use <= budget
    assert pr.peak_running >= 3                      # requests overlapped
    assert all(r.t_done >= r.t_admit >= r.t_arrival for r in res.values())


def test_oversized_request_rejected():
    pr = Probe(100)
    srv = serve.Server(100, workers=2, device=None, solve_fn=pr.solve, footprint_fn=pr.footprint)
    with pytest.raises(ValueError):
        srv.submit(_req(0, 101))
    srv.close()


def test_head_of_queue_is_not_starved():
    """A large request behind a stream of small ones is admitted once it has
    waited starvation_s: the small ones stop overtaking it."""
    budget = 1000
    pr = Probe(budget)
    srv = serve.Server(budget, workers=4, device=None, solve_fn=pr.solve,
                       footprint_fn=pr.footprint, starvation_s=0.05)
    srv.submit(_req(0, 600))
    srv.submit(_req(1, 600))                 # waits for memory
    for i in range(2, 40):
        srv.submit(_req(i, 100))
        time.sleep(0.005)
    res = srv.results(timeout=30)
    srv.close()
    assert len(res) == 40
    # the big request did not wait for the whole small stream
    assert res[1].t_admit < max(r.t_admit for r in res.values())


def test_failed_request_is_reported():
    def bad(req, device, stream):
        raise RuntimeError("boom")
    srv = serve.Server(10, workers=1, device=None, solve_fn=bad, footprint_fn=lambda r: 1)
    srv.submit(_req(0, 3))
    res = srv.results(timeout=10)
    srv.close()
    assert res[0].status == -99 and "boom" in res[0].error


def _gpu_requests():
    import workloads as wl
    reqs = []
    specs = [(101, 51, 4.0), (201, 101, 9.0), (401, 201, 10.0), (201, 101, 15.0),
             (101, 51, 18.0), (401, 201, 6.0), (201, 101, 3.0), (101, 51, 12.0)]
    for i, (nx, nz, fz) in enumerate(specs):
        w = wl.random_field_2d(nx, nz, 10.0, seed=1000 + i, freq_hz=fz, src=(nx // 2, 5))
        reqs.append(serve.Request(id=i, slowness=w.slowness, h=w.h, freq_hz=fz,
                                  source=w.source))
    return reqs


@pytest.mark.gpu
def test_mixed_stream_results_equal_alone():
    """Requests of different grids and frequencies submitted together overlap on
    four streams; each result has the bits of the same solve run alone, and
    meets the tolerance on the residual recomputed by the oracle's operator."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import operator as op
    reqs = _gpu_requests()
    srv = serve.Server(8 << 30, workers=4)
    for r in reqs:
        srv.submit(r)
    res = srv.results(timeout=300)
    srv.close()
    assert srv.max_concurrent >= 2
    dev = torch.device("cuda:0")
    for r in reqs:
        got = res[r.id]
        assert got.error is None and got.status == 0, got.error
        alone = serve.solve_one(r, dev, torch.cuda.current_stream())
        assert alone.iterations == got.iterations
        assert np.array_equal(alone.u, got.u)
        H = op.helmholtz(r.slowness, 2 * np.pi * r.freq_hz, r.alpha, r.h)
        b = op.weighted_rhs(r.source).ravel()
        assert np.linalg.norm(b - H @ got.u.ravel()) <= r.tol * (1 + 1e-6) * np.linalg.norm(b)


@pytest.mark.gpu
def test_footprint_covers_device_allocation():
    """The planned footprint is at least what the problem and its workspace take
    on the device (measured by the free device memory around the set-up)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import workloads as wl
    import paper_1712_08740_amd.hh as hh
    w = wl.grf_401x201()
    pb, wb = hh.footprint_bytes(w.shape, w.omega, w.slowness.max(), w.h)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    P = hh.Problem(torch.from_numpy(w.slowness).cuda(), w.omega, w.alpha, w.h)
    torch.cuda.synchronize()
    used_problem = free0 - torch.cuda.mem_get_info()[0]
    assert wb == P.workspace_bytes(w.restart)
    # the runtime rounds allocations up; the library's own buffers are all counted
    assert used_problem <= pb + (256 << 20)    # + the LU library's own scratch
    P.close()


def test_coarsest_limit_rule():
    """The serving dense limit: 8192, 16384 from 500k grid nodes, the
    request's own limit when it gives one, none in 1D."""
    def req(shape, **kw):
        return serve.Request(id=0, slowness=np.full(shape, 1 / 2000.0), h=10.0, freq_hz=10.0,
                             source=np.zeros(shape, complex), **kw)
    assert serve.coarsest_limit(req((401, 801))) == 8192
    assert serve.coarsest_limit(req((601, 1601))) == 16384
    assert serve.coarsest_limit(req((601, 1601), max_coarse=4096)) == 4096
    assert serve.coarsest_limit(req((1001,))) is None
