"""Stored oracle values (tests/golden/oracle_solves.json, written by
tests/golden/make_golden.py from oracle/ only) and the paper's printed
parameters (tests/golden/paper_parameters.json). A change in the oracle's
arithmetic shows up here first."""
import json
import os

import numpy as np

import workloads as wl
from oracle import solver, spectrum

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def test_layered_1d_well_reproduces_stored_solve():
    g = _load("oracle_solves.json")["layered_1d_well"]
    w = wl.layered_1d_well()
    res = solver.solve(w.slowness, w.omega, w.alpha, w.h, w.source, beta=w.beta,
                       tol=w.tol, restart=w.restart)
    assert res.iterations == g["iterations"]
    assert np.allclose(res.history, g["history"], rtol=1e-9, atol=1e-14)
    for i, (re, im) in g["samples"].items():
        assert abs(res.x.ravel()[int(i)] - complex(re, im)) <= 1e-9 * abs(complex(re, im)) + 1e-18


def test_grf_401x201_reproduces_stored_solve():
    g = _load("oracle_solves.json")["grf_401x201"]
    w = wl.grf_401x201()
    res = solver.solve(w.slowness, w.omega, w.alpha, w.h, w.source, beta=w.beta,
                       tol=w.tol, restart=w.restart)
    assert res.iterations == g["iterations"]
    assert np.allclose(res.history, g["history"], rtol=1e-8, atol=1e-14)


def test_paper_spectrum_parameters_put_spectrum_in_right_half_plane():
    """Fig. 2 with the paper's own parameters (30 Hz, beta1 = beta2 = 1)."""
    p = _load("paper_parameters.json")["spectrum_1d"]
    n, h, alpha = 201, 25.0, 0.01
    m = 1.0 / wl.layered_velocity_1d(n, h)
    mu = spectrum.preconditioned_eigenvalues(m, 2 * np.pi * p["freq_hz"], alpha,
                                             p["beta1"], p["beta2"], h)
    lam = spectrum.helmholtz_eigenvalues(m, 2 * np.pi * p["freq_hz"], alpha, h)
    assert lam.real.min() < 0 < mu.real.min()
