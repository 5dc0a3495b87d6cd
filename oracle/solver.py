"""The whole preconditioned solve (oracle; test infrastructure only).

Right-preconditioned GMRES on ``H u = W f`` (Eq. 3 and Eq. 7 with
``M_l = I``, ``M_r = M``), where ``M`` is the shifted Laplacian of Eq. 6 read
as ``-Lap - (beta1 - j beta2) k^2``. ``M^{-1}`` is applied

* ``"exact"``: exactly, by sparse LU of ``M`` (the 1D tridiagonal case);
* ``"mg"``:    approximately, by one V(2,2) cycle (``oracle.multigrid``);
* ``"none"``:  not at all (unpreconditioned GMRES, the paper's comparison).

1D problems use textbook GMRES and 2D problems flexible GMRES; with a fixed
linear preconditioner both produce the same iterates in exact arithmetic.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import operator as op
from .gmres import gmres, GmresResult
from .multigrid import VCycle, MAX_COARSE


def make_preconditioner(m, omega, beta1, beta2, h, kind: str, max_coarse: int = MAX_COARSE):
    if kind == "none":
        return None
    if kind == "exact":
        lu = spla.splu(op.shifted_laplace(m, omega, beta1, beta2, h).tocsc())
        return lu.solve
    if kind == "mg":
        return VCycle(m, omega, beta1, beta2, h, max_coarse=max_coarse)
    raise ValueError(kind)


def solve(m, omega, alpha, h, f, beta=(1.0, 0.5), tol=1e-6, restart=30,
          maxiter=2000, precond=None, flexible=None, keep_basis=False,
          max_coarse: int = MAX_COARSE) -> GmresResult:
    """Solve ``H u = W f``; returns the wavefield (grid-shaped) in ``result.x``."""
    m = np.asarray(m, dtype=np.float64)
    f = np.asarray(f, dtype=np.complex128)
    if precond is None:
        precond = "exact" if m.ndim == 1 else "mg"
    if flexible is None:
        flexible = m.ndim != 1
    H = op.helmholtz(m, omega, alpha, h)
    b = op.weighted_rhs(f)
    prec = make_preconditioner(m, omega, beta[0], beta[1], h, precond, max_coarse)
    res = gmres(lambda v: H @ v, b, tol, restart, maxiter, prec=prec,
                flexible=flexible, keep_basis=keep_basis)
    res.x = res.x.reshape(f.shape)
    return res
