"""Direct solve of ``H u = f`` by sparse LU, Eq. 4 (oracle; test infrastructure only).

The paper names LU factorisation as the direct method for small problems
(Eq. 4, Section "Data modelling") and uses it as the reference wavefield in
Fig. 3a and Fig. 6a. SciPy's SuperLU (``splu``) is the factorisation here.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import operator as op


def solve_direct(m, omega, alpha, h, f) -> np.ndarray:
    """``u = H^{-1} (W f)``, grid-shaped complex128."""
    f = np.asarray(f, dtype=np.complex128)
    H = op.helmholtz(m, omega, alpha, h)
    b = op.weighted_rhs(f)
    u = spla.splu(H.tocsc()).solve(b)
    return u.reshape(f.shape)


def solve_matrix(A, b) -> np.ndarray:
    """``A^{-1} b`` by SuperLU for an already assembled sparse matrix."""
    return spla.splu(A.tocsc()).solve(np.asarray(b, dtype=np.complex128))
