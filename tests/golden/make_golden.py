"""Writes the stored oracle values under tests/golden/ (calls only oracle/ and
the seeded input generators; nothing here comes from the GPU library).

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as wl                      # noqa: E402
from oracle import solver, direct           # noqa: E402


def summary(w, res, u_lu, samples):
    flat = res.x.ravel()
    return dict(
        workload=w.name, shape=list(w.shape), h=w.h, freq_hz=w.freq_hz, alpha=w.alpha,
        beta=list(w.beta), restart=w.restart, tol=w.tol,
        iterations=res.iterations, true_rel_res=res.true_rel_res,
        history=[float(x) for x in res.history],
        err_vs_lu=float(np.linalg.norm(res.x - u_lu) / np.linalg.norm(u_lu)),
        samples={str(i): [float(flat[i].real), float(flat[i].imag)] for i in samples},
    )


def main():
    out = {}
    w = wl.layered_1d_well()
    res = solver.solve(w.slowness, w.omega, w.alpha, w.h, w.source, beta=w.beta,
                       tol=w.tol, restart=w.restart)
    u = direct.solve_direct(w.slowness, w.omega, w.alpha, w.h, w.source)
    out["layered_1d_well"] = summary(w, res, u, [0, 100, 500, 1000])
    w = wl.grf_401x201()
    res = solver.solve(w.slowness, w.omega, w.alpha, w.h, w.source, beta=w.beta,
                       tol=w.tol, restart=w.restart)
    u = direct.solve_direct(w.slowness, w.omega, w.alpha, w.h, w.source)
    out["grf_401x201"] = summary(w, res, u, [0, 5 * 401 + 200, 100 * 401 + 300, 201 * 401 - 1])
    with open(os.path.join(HERE, "oracle_solves.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
