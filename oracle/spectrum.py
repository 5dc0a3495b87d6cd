"""Dense eigenvalues of ``H`` and of the preconditioned ``M^{-1} H`` (oracle;
test infrastructure only).

Fig. 2 of the paper shows the spectrum of the Helmholtz operator of the 1D
model at 30 Hz and of the preconditioned operator for ``beta1 = beta2 = 1``:
the preconditioned eigenvalues cluster on a circle and move away from the
origin and the negative real axis toward positive real values.

For ``beta1 = 1`` and ``beta2 > alpha`` the eigenvalues ``mu`` of
``M^{-1} H`` lie in the closed disc with centre ``(beta2 + alpha)/(2 beta2)``
and radius ``(beta2 - alpha)/(2 beta2)``: an eigenpair gives
``mu = (tau - sigma_H)/(tau - sigma_M)`` with
``tau = v^H A_0 v / v^H W K^2 v`` in the closed upper half plane, and that
Moebius map sends the upper half plane onto the disc.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import operator as op


def helmholtz_eigenvalues(m, omega, alpha, h) -> np.ndarray:
    return np.linalg.eigvals(op.helmholtz(m, omega, alpha, h).toarray())


def preconditioned_eigenvalues(m, omega, alpha, beta1, beta2, h) -> np.ndarray:
    """Eigenvalues of ``M^{-1} H`` (same as those of ``H M^{-1}``)."""
    H = op.helmholtz(m, omega, alpha, h).toarray()
    M = op.shifted_laplace(m, omega, beta1, beta2, h).toarray()
    return sla.eigvals(H, M)


def disc(alpha, beta2):
    """Centre and radius of the inclusion disc for ``beta1 = 1``."""
    return (beta2 + alpha) / (2.0 * beta2), (beta2 - alpha) / (2.0 * beta2)
