"""Benchmark: Helmholtz solves/s to a 1e-6 relative residual on one MI355X.

One step = one complete solve of the 401 x 201 (nx x nz) random-field workload
at 10 Hz (h = 10 m, alpha = 0.01, unit point source at (ix, iz) = (200, 5)):
right-preconditioned FGMRES(30), shifted Laplacian (1, 0.5) applied by one
V(2,2) omega-Jacobi multigrid cycle, complex128, tol 1e-6. The model, source
and preconditioner hierarchy are resident on the device before timing starts.

Prints one JSON line with throughput, per-solve latency percentiles, the
roofline figure of the dominant kernel (HIP-event durations of every launch
in the timed region, algorithmic bytes per launch from the kernel's byte
model) and the CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--workload grf_401x201|layered_1d_well]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# dense matrix-core peaks of the MI355X (TFLOP/s)
MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
METRIC = "Helmholtz solves/s to 1e-6 residual; HBM GB/s; p50/p99 latency vs plain"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="grf_401x201",
                    choices=["grf_401x201", "layered_1d_well", "grf_1201x401",
                             "grf_801x301_batch", "serving", "stream_probe"],
                    help="grf_801x301_batch: 32 top-row sources x 4 frequencies, one batched "
                         "solve of 32 sources per frequency (a step = all 128 solves)")
    ap.add_argument("--max-coarse", type=int, default=None,
                    help="dense limit of the coarsest multigrid grid (default 4096; the batched "
                         "workload uses 16384)")
    ap.add_argument("--precision", default="f64", choices=["f64", "mixed"],
                    help="mixed: the preconditioner in complex64 inside the FP64 FGMRES")
    ap.add_argument("--kernel", default="auto",
                    help="kernel class for the roofline figure; 'auto' (default) times every "
                         "class over one warm-up solve and takes the one with the most device time")
    ap.add_argument("--tiles", default=None, choices=["auto", "default"],
                    help="tile shapes of the multigrid legs: 'auto' times every shape on the "
                         "workload's hierarchy during set-up (hh_autotune), 'default' keeps the "
                         "fixed rule. Unset: 'auto' for the batched workload (measured faster), "
                         "'default' for single sources (the tuner's picks there are within the "
                         "timing noise and may differ from run to run)")
    ap.add_argument("--batch-streams", type=int, default=1,
                    help="batched workload: the frequencies' batches run concurrently on this "
                         "many streams, one host thread each (default 1: one after another, so "
                         "that the roofline times each kernel without contention; 2-4 streams "
                         "measured 2% more solves/s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-checks", action="store_true",
                    help="skip the comparisons run after the timed region (error against the "
                         "FP64 solve, plain FP64 throughput): for profiler runs whose kernel "
                         "classes should hold the timed workload's launches only")
    ap.add_argument("--requests", type=int, default=200,
                    help="serving: requests in the Poisson stream (mean 200/s)")
    ap.add_argument("--serve-workers", type=int, default=4,
                    help="serving: concurrent streams")
    ap.add_argument("--serve-budget-gib", type=float, default=128.0,
                    help="serving: device memory budget for admitted requests")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the solves, copy a buffer of this many MiB once on the device "
                         "(a plain copy kernel of known size, to scale hardware byte counters)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="wall-clock budget of the CPU oracle sample")
    a = ap.parse_args()
    if a.tiles is None:
        a.tiles = "auto" if a.workload == "grf_801x301_batch" else "default"
    return a


def measured_traffic(workload_name: str, kernel: str):
    """HBM bytes per launch of a kernel class from the committed --pmc summaries
    (profiles/hbm_traffic_*.md), or None when there is none or the kernel's
    sources changed since the counters were taken."""
    import glob
    sys.path.insert(0, ROOT)
    from profile_summary import source_digest
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.md"))):
        text = open(path).read()
        if "```json" not in text:
            continue
        block = text.split("```json", 1)[1].split("```", 1)[0]
        entry = json.loads(block).get(workload_name, {}).get(kernel)
        if entry and entry["digest"] == source_digest(kernel):
            return entry["bytes_per_launch"]
    return None


def workload(name):
    import workloads as wl
    return {"grf_401x201": wl.grf_401x201, "layered_1d_well": wl.layered_1d_well,
            "grf_1201x401": wl.grf_1201x401}[name]()


def cpu_baseline(w, budget_s: float, gpu_iterations: int):
    """The oracle (``oracle.solver.solve``, unchanged) on the same workload,
    BLAS pinned to one thread. Small grids: complete solves repeated until the
    time budget is spent. Large grids (a complete oracle solve takes minutes):
    two truncated solves (10 and 30 iterations, set-up included) give the
    set-up time and the time per iteration, and one solve is priced at the
    set-up plus the iteration count the GPU solve took (the oracle takes the
    same count, +-1)."""
    from threadpoolctl import threadpool_limits
    from oracle import solver

    def run(maxiter):
        t = time.perf_counter()
        r = solver.solve(w.slowness, w.omega, w.alpha, w.h, w.source, beta=w.beta,
                         tol=w.tol, restart=w.restart, maxiter=maxiter)
        return time.perf_counter() - t, r

    with threadpool_limits(limits=1):
        if w.slowness.size <= 200_000:
            n, its, t0 = 0, None, time.perf_counter()
            while True:
                _, r = run(2000)
                n += 1
                its = r.iterations
                el = time.perf_counter() - t0
                if el >= budget_s or n >= 50:
                    break
            return {"value": n / el, "unit": "solves/s", "cores": 1, "kind": "oracle",
                    "sample": f"{n} complete oracle solves of the same workload (set-up "
                              f"included, {its} iterations each) in {el:.1f} s, NumPy/SciPy "
                              f"FP64, 1 thread"}
        t10, _ = run(10)
        t30, _ = run(30)
        per_it = (t30 - t10) / 20.0
        setup = max(t10 - 10 * per_it, 0.0)
        est = setup + gpu_iterations * per_it
        return {"value": 1.0 / est, "unit": "solves/s", "cores": 1, "kind": "oracle",
                "sample": f"oracle truncated at 10 and 30 iterations ({t10:.1f} s, {t30:.1f} s, "
                          f"set-up included): {setup:.1f} s set-up + {per_it:.2f} s/iteration, "
                          f"priced at {gpu_iterations} iterations = {est:.1f} s per solve; "
                          f"NumPy/SciPy FP64, 1 thread"}


def cpu_baseline_batch(slow, sources, freqs, budget_s: float, its_by_freq, max_coarse: int):
    """The oracle on the batched workload: per frequency, two truncated solves
    of one source (10 and 30 iterations) give the set-up and per-iteration
    time; each of the 32 sources of that frequency is priced at the iteration
    count the GPU took for it (set-up once per frequency: the oracle builds its
    hierarchy per solve, so this favours the oracle)."""
    from threadpoolctl import threadpool_limits
    from oracle import solver
    total, parts = 0.0, []
    with threadpool_limits(limits=1):
        for fz, its in zip(freqs, its_by_freq):
            f = np.zeros(slow.shape, complex)
            f[sources[0][1], sources[0][0]] = 1.0
            om = 2 * np.pi * fz

            def run(maxiter):
                t = time.perf_counter()
                solver.solve(slow, om, 0.01, 10.0, f, tol=1e-6, restart=30, maxiter=maxiter,
                             max_coarse=max_coarse)
                return time.perf_counter() - t
            t10, t30 = run(10), run(30)
            per_it = (t30 - t10) / 20.0
            setup = max(t10 - 10 * per_it, 0.0)
            cost = setup + per_it * float(np.sum(its))
            total += cost
            parts.append(f"{fz} Hz: {setup:.1f} s + {per_it:.3f} s/it x {int(np.sum(its))} its")
    n = len(freqs) * len(sources)
    return {"value": n / total, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle truncated at 10 and 30 iterations per frequency, priced at the "
                      f"GPU's per-source iteration counts ({'; '.join(parts)}) = {total:.0f} s "
                      f"for {n} solves; NumPy/SciPy FP64, 1 thread"}


def _tile_names(hh, tiles, mode):
    """Tile shapes per level with legs, as 'down/up' (the fixed rule: 'default')."""
    if mode != "auto":
        return "default"
    def name(shapes, t):
        return "default" if t < 0 else shapes[t]
    return [f"{name(hh.TILE_DOWN_SHAPES, d)}/{name(hh.TILE_UP_SHAPES, u)}" for d, u in tiles]


def main_batch(a, hh, torch, dev):
    import workloads as wl
    slow, sources, freqs = wl.grf_801x301_sources()
    nz, nx = slow.shape
    F = np.zeros((len(sources), nz, nx), complex)
    for i, (ix, iz) in enumerate(sources):
        F[i, iz, ix] = 1.0
    Ft = torch.from_numpy(F).to(dev)
    m = torch.from_numpy(slow).to(dev)
    mixed = a.precision == "mixed"
    restart, tol = 30, 1e-6
    t_setup = time.perf_counter()
    max_coarse = a.max_coarse or 16384
    probs = [hh.Problem(m, 2 * np.pi * fz, 0.01, 10.0, max_coarse=max_coarse) for fz in freqs]
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    t_tune = time.perf_counter()
    tiles = [P.autotune(precond_f32=mixed, nrhs=len(sources)) if a.tiles == "auto" else []
             for P in probs]
    t_tune = time.perf_counter() - t_tune
    wss = [torch.empty(P.workspace_bytes_batch(restart, len(sources)), dtype=torch.uint8,
                       device=dev) for P in probs]
    Us = [torch.empty_like(Ft) for _ in probs]
    # one stream (default priority) and host thread per frequency: the batches
    # are independent problems, so their kernels may overlap on the device
    nstreams = max(1, min(a.batch_streams, len(probs)))
    streams = [torch.cuda.Stream(device=dev) for _ in range(nstreams)]
    torch.cuda.synchronize()

    def solve_group(g):
        return [P.solve_batch(Ft, tol=tol, restart=restart, max_iters=2000, precond_f32=mixed,
                              U=Us[i], workspace=wss[i], stream=streams[g])
                for i, P in enumerate(probs) if i % nstreams == g]

    pool = None
    if nstreams > 1:
        from concurrent.futures import ThreadPoolExecutor
        pool = ThreadPoolExecutor(max_workers=nstreams)

    def one():
        if pool is None:
            return solve_group(0)
        groups = list(pool.map(solve_group, range(nstreams)))
        out = [None] * len(probs)
        for g, rs in enumerate(groups):
            for j, r in enumerate(rs):
                out[g + j * nstreams] = r
        return out

    for _ in range(a.warmup):
        one()
    share = {}
    for k in hh.KERNEL_IDS:
        if k == "none":
            continue
        for P in probs:
            P.kernel_timer_start(k)
        one()
        tot = 0.0
        for P in probs:
            n_k, ms_k, _ = P.kernel_timer_read()
            tot += ms_k
            P.kernel_timer_start("none")
        if tot > 0:
            share[k] = tot
    kernel = max(share, key=share.get) if a.kernel == "auto" else a.kernel
    for P in probs:
        P.kernel_timer_start(kernel)
    torch.cuda.synchronize()
    lat, its, res = [], None, []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        t1 = time.perf_counter()
        rs = one()
        lat.append(time.perf_counter() - t1)
        its = [r.iterations for r in rs]
        for r in rs:
            res.append(float(r.true_rel_res.max()))
            if r.overall != hh.HH_OK or r.true_rel_res.max() > tol:
                print("batched solve did not converge", file=sys.stderr)
                sys.exit(1)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launches = kms = kbytes = kflops = 0
    for P in probs:
        n_k, ms_k, b_k = P.kernel_timer_read()
        launches += n_k
        kms += ms_k
        kbytes += b_k
        # the batched coarsest product: 8 real flops per complex multiply-add,
        # nc^2 of them per source
        nz_c, nx_c = P.level_info(P.num_levels - 1)[0]
        kflops += n_k * 8.0 * float(nz_c * nx_c) ** 2 * len(sources)
        P.kernel_timer_start("none")
    precision = None
    if mixed and not a.no_checks:
        # after the timed region: every source again with the complex128 cycle
        diffs = []
        for i, P in enumerate(probs):
            u32 = Us[i].clone()
            r64 = P.solve_batch(Ft, tol=tol, restart=restart, max_iters=2000, U=Us[i],
                                workspace=wss[i])
            d = torch.linalg.vector_norm((u32 - r64.u).reshape(len(sources), -1), dim=1)
            d = d / torch.linalg.vector_norm(r64.u.reshape(len(sources), -1), dim=1)
            diffs.append(float(d.max()))
        torch.cuda.synchronize()
        precision = {"max_rel_diff_vs_fp64_solve_by_freq": diffs,
                     "reference": "hh_solve_batch with the complex128 preconditioner, same "
                                  "tol and restart"}
    # the plain solver on the same sources: single sources one at a time with
    # the complex128 cycle and the default dense coarsest limit (8 sources per
    # frequency; problems set up outside the timing, as the batch's), after the
    # timed region
    sample = list(range(0, len(sources), max(1, len(sources) // 8)))[:8]
    if a.no_checks:
        sample = []
    plain_probs = [hh.Problem(m, 2 * np.pi * fz, 0.01, 10.0) for fz in freqs] if sample else []
    plain_ws = [Q.workspace(restart) for Q in plain_probs]
    plain_its = []
    torch.cuda.synchronize()
    t_plain = time.perf_counter()
    for Q, ws1 in zip(plain_probs, plain_ws):
        for i in sample:
            r1 = Q.solve(Ft[i], tol=tol, restart=restart, max_iters=2000, workspace=ws1)
            if r1.status != hh.HH_OK:
                print("plain solve did not converge", file=sys.stderr)
                sys.exit(1)
            plain_its.append(r1.iterations)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t_plain
    plain = None if not plain_its else {
             "solves_per_s": len(plain_its) / t_plain,
             "iterations_min_max": [min(plain_its), max(plain_its)],
             "sample": f"{len(sample)} sources per frequency, one hh_solve each, complex128 "
                       "preconditioner, default dense coarsest limit, same tol and restart"}
    del plain_probs, plain_ws
    achieved = (kbytes / (kms * 1e-3)) / 1e9 if kms > 0 else 0.0
    if kernel == "gemv":
        # a dense contraction on the matrix cores: priced against the MFMA peak
        peak = MFMA_PEAK_TFLOPS["f32" if mixed else "f64"]
        achieved_tf = (kflops / (kms * 1e-3)) / 1e12 if kms > 0 else 0.0
        roof = {"bound": "mfma", "kernel": kernel, "achieved": achieved_tf, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved_tf / peak,
                "hbm_gbs": achieved, "algorithmic_flops_per_launch": kflops / max(launches, 1)}
    else:
        roof = {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS}
    n_solves = len(freqs) * len(sources)
    out = {
        "metric": METRIC,
        "value": a.steps * n_solves / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128+c64" if mixed else "c128",
        "data": "synthetic",
        "config": {
            "workload": "grf2d_801x301_s4_32src_x_4freq",
            "grid_nx_nz": [nx, nz], "h_m": 10.0, "freq_hz": freqs, "alpha": 0.01,
            "beta": [1.0, 0.5], "tol": tol, "restart": restart, "sources_per_batch": len(sources),
            "solves_per_step": n_solves, "max_coarse": max_coarse, "streams": nstreams,
            "precond": "V(2,2) omega-Jacobi, Galerkin coarse operators, dense coarsest inverse"
                       + (", complex64 inside FP64 FGMRES" if mixed else ", complex128"),
            "levels_nz_nx": [[list(P.level_info(l)[0]) for l in range(P.num_levels)]
                             for P in probs[:1]][0],
            "iterations_min_max_by_freq": [[int(i.min()), int(i.max())] for i in its],
            "true_rel_res_max": max(res),
            "setup_ms": 1e3 * t_setup,
            "precision_check": precision,
            "plain_fp64_one_at_a_time": plain,
            "tiles_down_up_by_freq": [_tile_names(hh, t, a.tiles) for t in tiles],
            "autotune_ms": 1e3 * t_tune,
        },
        "latency_ms": {"p50_step": float(np.percentile(lat, 50) * 1e3),
                       "p99_step": float(np.percentile(lat, 99) * 1e3),
                       "plain": "a step is the 128 solves; the plain one-at-a-time solver is "
                                "bench.py without --workload"},
        "roofline": {
            **roof,
            "traffic": measured_traffic("grf2d_801x301_batch" + ("_mixed" if mixed else ""),
                                        kernel),
            "launches": int(launches), "avg_launch_us": 1e3 * kms / max(launches, 1),
            "algorithmic_bytes_per_launch": kbytes / max(launches, 1),
            "device_ms_per_step_by_kernel": {k: round(v, 3) for k, v in
                                             sorted(share.items(), key=lambda kv: -kv[1])},
        },
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batch(slow, sources, freqs, a.cpu_seconds, its,
                                                 max_coarse)
    print(json.dumps(out), flush=True)


def main_serving(a, hh, torch, dev):
    """A Poisson stream of single-source requests (grids 201x101 .. 1601x601,
    3-20 Hz, per-request seeded models) through the request loop: solves/s over
    the stream and p50/p99 latency from arrival to result."""
    import workloads as wl
    from paper_1712_08740_amd import serve
    stream = wl.serving_stream(n_requests=a.requests, rate_hz=200.0, seed=5)
    reqs = []
    t_gen = time.perf_counter()
    for r in stream:
        w = wl.random_field_2d(r["nx"], r["nz"], 10.0, seed=r["seed"], freq_hz=r["freq_hz"],
                               src=r["src"])
        reqs.append((r["t_arrival"], serve.Request(
            id=r["id"], slowness=w.slowness, h=w.h, freq_hz=r["freq_hz"], source=w.source,
            precond_f32=a.precision == "mixed")))
    t_gen = time.perf_counter() - t_gen
    # warm-up: one small request through the library (kernel loading, LU library)
    serve.solve_one(reqs[0][1], dev, torch.cuda.current_stream())
    srv = serve.Server(int(a.serve_budget_gib * (1 << 30)), workers=a.serve_workers)
    t0 = time.perf_counter()
    for t_arr, rq in reqs:
        wait = t_arr - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        srv.submit(rq)
    res = srv.results(timeout=3600)
    wall = time.perf_counter() - t0
    srv.close()
    results = [res[i] for i in sorted(res)]
    st = serve.summarize(results, wall)
    by_grid = {}
    for (_, rq), r in zip(reqs, results):
        key = f"{rq.slowness.shape[1]}x{rq.slowness.shape[0]}"
        by_grid.setdefault(key, []).append(r.latency * 1e3)
    precision = plain = None
    if a.precision == "mixed" and not a.no_checks:
        # after the stream: every request again with the complex128 cycle
        import dataclasses
        diffs, worst = [], None
        torch.cuda.synchronize()
        t_plain = time.perf_counter()
        for (_, rq), r in zip(reqs, results):
            ref = serve.solve_one(dataclasses.replace(rq, precond_f32=False), dev,
                                  torch.cuda.current_stream())
            d = float(np.linalg.norm(r.u - ref.u) / np.linalg.norm(ref.u))
            diffs.append(d)
            if worst is None or d > worst["rel_diff"]:
                worst = {"rel_diff": d, "grid_nx_nz": [rq.slowness.shape[1], rq.slowness.shape[0]],
                         "freq_hz": rq.freq_hz, "iterations_c64": r.iterations,
                         "iterations_c128": ref.iterations,
                         "true_rel_res_c64": r.true_rel_res, "true_rel_res_c128": ref.true_rel_res}
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t_plain
        plain = {"solves_per_s": len(diffs) / t_plain,
                 "what": "the same requests one at a time, set-up included, complex128 "
                         "preconditioner, on one stream, back to back (no arrival gaps); "
                         "includes copying each result to the host"}
        precision = {"rel_diff_vs_fp64_solve_max": max(diffs),
                     "rel_diff_vs_fp64_solve_median": float(np.median(diffs)),
                     "requests": len(diffs), "largest": worst,
                     "reference": "each request solved again with the complex128 "
                                  "preconditioner, same tol and restart"}
    out = {
        "metric": METRIC,
        "value": st["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1, "steps": len(results), "warmup": 1,
        "ms_per_step": 1e3 * wall / len(results),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128+c64" if a.precision == "mixed" else "c128",
        "data": "synthetic",
        "config": {"workload": f"serving_poisson200_{a.requests}req",
                   "grids_nx_nz": [list(g) for g in wl.SERVING_GRIDS], "freq_hz": [3.0, 20.0],
                   "h_m": 10.0, "alpha": 0.01, "tol": 1e-6, "restart": 30,
                   "workers": a.serve_workers, "budget_gib": a.serve_budget_gib,
                   "converged": st["converged"], "max_iterations": st["max_iterations"],
                   "model_generation_s": t_gen, "precision_check": precision,
                   "plain_fp64_one_at_a_time": plain},
        "latency_ms": {"p50": st["latency_p50_ms"], "p99": st["latency_p99_ms"],
                       "queue_p50": st["queue_p50_ms"], "queue_p99": st["queue_p99_ms"],
                       "p50_by_grid": {k: float(np.percentile(v, 50)) for k, v in by_grid.items()},
                       "plain": "bench.py without --workload is the plain one-at-a-time solver"},
        "peak_admitted_gib": srv.peak_in_use / 2 ** 30,
        "max_concurrent": srv.max_concurrent,
        "roofline": None,
    }
    print(json.dumps(out), flush=True)


def main_stream_probe(torch, dev):
    """The HBM bandwidth plain streaming kernels reach on this device (PyTorch's
    own copy, sum and axpy over 1 GiB float64 vectors, best of five, events on
    the stream): the practical ceiling beside the 8 TB/s peak."""
    n = (1 << 30) // 8
    x = torch.ones(n, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    for name, fn, nbytes in (("copy", lambda: y.copy_(x), 16 * n),
                             ("sum", lambda: x.sum(), 8 * n),
                             ("axpy", lambda: y.add_(x, alpha=2.0), 24 * n)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(5):
            s0.record()
            fn()
            s1.record()
            torch.cuda.synchronize()
            best = min(best, s0.elapsed_time(s1))
        out[name] = {"GB/s": nbytes / (best * 1e-3) / 1e9, "ms": best, "bytes": nbytes}
    print(json.dumps({"metric": "device streaming bandwidth (practical ceiling)",
                      "peak_GB/s": HBM_PEAK_GBS, "kernels": out}), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              "(the solver does not shard across GPUs).", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    import torch
    import paper_1712_08740_amd.hh as hh

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    if a.copy_probe_mib > 0:
        src = torch.ones(a.copy_probe_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.workload == "stream_probe":
        return main_stream_probe(torch, dev)
    if a.workload == "grf_801x301_batch":
        return main_batch(a, hh, torch, dev)
    if a.workload == "serving":
        return main_serving(a, hh, torch, dev)
    w = workload(a.workload)
    stream = torch.cuda.current_stream()
    m = torch.from_numpy(w.slowness).to(dev)
    f = torch.from_numpy(w.source).to(dev)
    t_setup = time.perf_counter()
    P = hh.Problem(m, w.omega, w.alpha, w.h, beta=w.beta, max_coarse=a.max_coarse)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    ws = P.workspace(w.restart)
    u = torch.empty_like(f)

    mixed = a.precision == "mixed"
    t_tune = time.perf_counter()
    tiles = P.autotune(precond_f32=mixed) if a.tiles == "auto" else []
    t_tune = time.perf_counter() - t_tune

    def one():
        return P.solve(f, tol=w.tol, restart=w.restart, max_iters=2000, u=u, workspace=ws,
                       precond_f32=mixed)

    for _ in range(a.warmup):
        one()
    # device time per solve of every kernel class (one solve per class)
    share = {}
    for k in hh.KERNEL_IDS:
        if k == "none":
            continue
        P.kernel_timer_start(k)
        one()
        n_k, ms_k, _ = P.kernel_timer_read()
        if n_k:
            share[k] = ms_k
    P.kernel_timer_start("none")
    kernel = max(share, key=share.get) if a.kernel == "auto" else a.kernel
    P.kernel_timer_start(kernel)
    torch.cuda.synchronize()
    lat = []
    its = []
    res = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        t1 = time.perf_counter()
        r = one()
        lat.append(time.perf_counter() - t1)
        its.append(r.iterations)
        res.append(r.true_rel_res)
        if r.status != hh.HH_OK or r.true_rel_res > w.tol:
            print(f"solve did not converge: status {r.status} res {r.true_rel_res}",
                  file=sys.stderr)
            sys.exit(1)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launches, kms, kbytes = P.kernel_timer_read()
    P.kernel_timer_start("none")
    precision = None
    if mixed and not a.no_checks:
        # after the timed region: the same solve with the complex128 cycle, the
        # FP64 reference the complex64 result is stated against
        u32 = u.clone()
        r64 = P.solve(f, tol=w.tol, restart=w.restart, max_iters=2000, workspace=ws)
        precision = {
            "rel_diff_vs_fp64_solve": float(torch.linalg.vector_norm(u32 - r64.u)
                                            / torch.linalg.vector_norm(r64.u)),
            "fp64_iterations": int(r64.iterations),
            "true_rel_res_fp64_recomputed": float(max(res)),
            "reference": "hh_solve with the complex128 preconditioner, same tol and restart "
                         "(the parity tests pin it to the oracle's LU solution within 1e-6)"}

    comparison = None
    if not a.no_checks:
        # after the timed region: the paper's comparison, GMRES on the Helmholtz
        # operator itself (no preconditioner), same restart, capped iterations
        cap = 4000
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rn = P.solve(f, tol=w.tol, restart=w.restart, max_iters=cap, workspace=ws,
                     no_precond=True, hist_cap=0)
        torch.cuda.synchronize()
        comparison = {
            "unpreconditioned_gmres": {
                "iterations": int(rn.iterations), "status": int(rn.status),
                "converged": rn.status == hh.HH_OK, "true_rel_res": float(rn.true_rel_res),
                "ms": 1e3 * (time.perf_counter() - t1), "max_iters": cap},
            "preconditioned_iterations": int(np.median(its))}

    avg_us = 1e3 * kms / max(launches, 1)
    achieved = (kbytes / (kms * 1e-3)) / 1e9 if kms > 0 else 0.0
    # whole-solve effective bandwidth from the byte model of all kernels is not
    # reported as HBM: the working set of this workload is cache-resident.
    levels = [P.level_info(l)[0] for l in range(P.num_levels)]
    out = {
        "metric": METRIC,
        "value": a.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128+c64" if mixed else "c128",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "grid_nx_nz": [int(w.shape[-1]), int(w.shape[0]) if len(w.shape) == 2 else 1],
            "h_m": w.h, "freq_hz": w.freq_hz, "alpha": w.alpha, "beta": list(w.beta),
            "tol": w.tol, "restart": w.restart,
            "precond": ("V(2,2) omega-Jacobi (0.8 where omega*max(m)*h < 2, else 0.5), Galerkin "
                        "coarse operators, dense coarsest inverse"
                        if len(w.shape) == 2 else "exact tridiagonal (PCR)")
                       + (", complex64 inside FP64 FGMRES" if mixed else ", complex128"),
            "levels_nz_nx": levels,
            "iterations": int(np.median(its)),
            "true_rel_res_max": float(max(res)),
            "setup_ms": 1e3 * t_setup,
            "precision_check": precision,
            "precond_comparison": comparison,
            "tiles_down_up": _tile_names(hh, tiles, a.tiles),
            "autotune_ms": 1e3 * t_tune,
        },
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                       "p99": float(np.percentile(lat, 99) * 1e3),
                       "plain": "this is the plain FP64 one-request-at-a-time solver"},
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(w.name + ("_mixed" if mixed else ""), kernel),
            "launches": int(launches),
            "avg_launch_us": avg_us,
            "algorithmic_bytes_per_launch": kbytes / max(launches, 1),
            "device_ms_per_solve_by_kernel": {k: round(v, 4) for k, v in
                                              sorted(share.items(), key=lambda kv: -kv[1])},
        },
    }
    if rank == 0 and not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_seconds, int(np.median(its)))
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
