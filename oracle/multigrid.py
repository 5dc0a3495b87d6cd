"""One multigrid V-cycle on the shifted Laplacian as ``M^{-1}`` (oracle;
test infrastructure only).

The paper applies ``P^{-1}`` of Eq. 6-7 but does not say how it is inverted.
For 2D grids this oracle defines the approximate inverse as one V(2,2) cycle:

* levels: a grid dimension of ``n`` nodes with spacing ``h`` is halved to
  ``(n-1)/2 + 1`` nodes (spacing ``2h``) when ``n-1`` is even,
  ``(n-1)/2 >= 2`` and either the coarse grid still has at least two nodes per
  shortest wavelength, ``omega * max(m) * 2h <= pi``, or the current grid has
  more than ``max_coarse`` (4096) nodes (too many for the direct coarsest
  solve); each dimension is treated on its own (semi-coarsening once one
  stops) until neither halves;
* prolongation ``P``: (bi)linear interpolation in the halved dimensions;
  restriction ``R = P^T / 2^{d_c}`` (``d_c`` = number of halved dimensions;
  full weighting ``[1 2 1; 2 4 2; 1 2 1]/16`` at interior 2D nodes);
* the finest operator is ``M`` itself; each coarser operator is the Galerkin
  product ``M_{l+1} = R_l M_l P_l`` (a 9-point stencil in 2D);
* smoother: omega-Jacobi, ``x <- x + omega_J D^{-1} (b - M x)`` with
  ``D = diag(M)``; ``omega_J = 0.8`` on levels with
  ``omega * max(m) * max(h_x, h_z) < 2`` and 0.5 on coarser (under-resolved)
  levels, where 0.8 no longer damps; 2 sweeps before and 2 after the coarse
  correction, starting from ``x = 0`` on every level;
* the coarsest level is solved directly (SuperLU).
"""
from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import operator as op


MAX_COARSE = 4096        # largest grid solved directly on the coarsest level
KH_SMOOTH = 2.0          # omega_J = 0.8 below this k*h, 0.5 at and above


def coarsen_shape(shape, spacing, kmax: float,
                  max_coarse: int = MAX_COARSE) -> Tuple[Tuple[int, ...], Tuple[bool, ...]]:
    """Next coarser grid shape and which dimensions were halved.

    ``kmax = omega * max(m)`` is the largest wavenumber of the model.
    """
    big = int(np.prod(shape)) > max_coarse
    new, halved = [], []
    for n, h in zip(shape, spacing):
        if (n - 1) % 2 == 0 and (n - 1) // 2 >= 2 and (kmax * 2.0 * h <= np.pi or big):
            new.append((n - 1) // 2 + 1)
            halved.append(True)
        else:
            new.append(n)
            halved.append(False)
    return tuple(new), tuple(halved)


def level_shapes(shape, spacing, kmax: float, max_coarse: int = MAX_COARSE) -> List[Tuple[int, ...]]:
    shapes = [tuple(shape)]
    sp_ = tuple(spacing)
    while True:
        nxt, halved = coarsen_shape(shapes[-1], sp_, kmax, max_coarse)
        if not any(halved):
            return shapes
        shapes.append(nxt)
        sp_ = tuple(h * (2.0 if hv else 1.0) for h, hv in zip(sp_, halved))


def interpolation_1d(n_fine: int, halved: bool) -> sp.csr_matrix:
    """Linear interpolation from ``(n_fine-1)/2+1`` coarse nodes (or identity)."""
    if not halved:
        return sp.identity(n_fine, dtype=np.float64, format="csr")
    n_c = (n_fine - 1) // 2 + 1
    P = sp.lil_matrix((n_fine, n_c), dtype=np.float64)
    for i in range(n_fine):
        if i % 2 == 0:
            P[i, i // 2] = 1.0
        else:
            P[i, i // 2] = 0.5
            P[i, i // 2 + 1] = 0.5
    return P.tocsr()


def prolongation(fine_shape, halved) -> sp.csr_matrix:
    """Tensor-product (bi)linear interpolation matrix, coarse -> fine."""
    mats = [interpolation_1d(n, hv) for n, hv in zip(fine_shape, halved)]
    P = mats[0]
    for Mk in mats[1:]:
        P = sp.kron(P, Mk, format="csr")     # row-major: first axis slowest
    return P.tocsr()


def restriction(fine_shape, halved) -> sp.csr_matrix:
    """``R = P^T / 2^{d_c}``."""
    dc = sum(1 for hv in halved if hv)
    return (prolongation(fine_shape, halved).T / float(2 ** dc)).tocsr()


@dataclasses.dataclass
class Level:
    shape: Tuple[int, ...]
    spacing: Tuple[float, ...]
    M: sp.csr_matrix
    Dinv: np.ndarray
    omega_j: float = 0.8             # Jacobi weight on this level
    P: sp.csr_matrix = None          # prolongation from the next coarser level
    R: sp.csr_matrix = None          # restriction to the next coarser level
    lu: object = None                # coarsest level only


class VCycle:
    """V(nu1, nu2) cycle for ``M = A_{beta1 - j beta2}`` on a 2D (or 1D) grid."""

    def __init__(self, m, omega, beta1, beta2, h, nu1: int = 2, nu2: int = 2,
                 omega_j: float = 0.8, omega_j_coarse: float = 0.5,
                 max_coarse: int = MAX_COARSE):
        m = np.asarray(m, dtype=np.float64)
        ndim = m.ndim
        spacing = (float(h),) * ndim if np.isscalar(h) else tuple(float(x) for x in h)
        sigma = beta1 - 1j * beta2
        kmax = omega * float(m.max())
        self.nu1, self.nu2 = nu1, nu2
        self.levels: List[Level] = []
        shape, cur_h = m.shape, spacing
        M = op.assemble(m, omega, sigma, spacing)
        while True:
            wj = omega_j if kmax * max(cur_h) < KH_SMOOTH else omega_j_coarse
            lev = Level(shape=shape, spacing=cur_h, M=M, Dinv=1.0 / M.diagonal(), omega_j=wj)
            self.levels.append(lev)
            nxt, halved = coarsen_shape(shape, cur_h, kmax, max_coarse)
            if not any(halved):
                lev.lu = spla.splu(M.tocsc())
                break
            lev.P = prolongation(shape, halved)
            lev.R = restriction(shape, halved)
            M = (lev.R @ M @ lev.P).tocsr()            # Galerkin coarse operator
            shape = nxt
            cur_h = tuple(hh * (2.0 if hv else 1.0) for hh, hv in zip(cur_h, halved))

    @property
    def shapes(self):
        return [lev.shape for lev in self.levels]

    def jacobi(self, lev: Level, x, b):
        """One omega-Jacobi sweep ``x + omega_J D^{-1} (b - M x)``."""
        return x + lev.omega_j * lev.Dinv * (b - lev.M @ x)

    def cycle(self, l: int, b: np.ndarray) -> np.ndarray:
        lev = self.levels[l]
        if l == len(self.levels) - 1:
            return lev.lu.solve(b)
        x = np.zeros_like(b)
        for _ in range(self.nu1):
            x = self.jacobi(lev, x, b)
        bc = lev.R @ (b - lev.M @ x)
        x = x + lev.P @ self.cycle(l + 1, bc)
        for _ in range(self.nu2):
            x = self.jacobi(lev, x, b)
        return x

    def __call__(self, v: np.ndarray) -> np.ndarray:
        return self.cycle(0, np.asarray(v, dtype=np.complex128))

    def as_matrix(self) -> np.ndarray:
        """Dense matrix of the (linear) cycle, one column per unit vector; tiny grids only."""
        N = self.levels[0].M.shape[0]
        B = np.empty((N, N), dtype=np.complex128)
        e = np.zeros(N, dtype=np.complex128)
        for i in range(N):
            e[:] = 0.0
            e[i] = 1.0
            B[:, i] = self(e)
        return B
