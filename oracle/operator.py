"""Discrete Helmholtz-type operator ``A_sigma`` (oracle; test infrastructure only).

The paper solves the constant-density damped Helmholtz equation
``-Lap u - omega^2 m^2 (1 - j alpha) u = f`` (Eq. 2, slowness ``m = 1/c``,
wavenumber ``k = omega m``) with a first-order absorbing boundary
(Section "Data modelling"), written as ``H u = f`` (Eq. 3). It prints no
discretisation. The reading used here:

* second-order centred differences (3-point in 1D, 5-point in 2D);
* boundary condition ``du/dn + j k u = 0`` (the sign follows from the
  damping sign of Eq. 2, i.e. an ``exp(+j omega t)`` time convention), put in
  with a centred ghost point that is then eliminated;
* every boundary row is multiplied by 1/2 per boundary axis (1/2 on edges,
  1/4 at corners) so that the matrix is exactly complex-symmetric; the same
  diagonal row weights ``W`` multiply the right-hand side: ``A u = W f``.

For a shift coefficient ``sigma`` and a d-dimensional grid (axes in storage
order; 2D is ``(z, x)`` with x fastest) the row of node ``p`` is

  sum over axes a:  (prod_{b != a} w_b) / h_a^2 * sum_{q = a-neighbours} (u_p - u_q)
                  + j k_p * e_a * (prod_{b != a} w_b) / h_a * u_p
  - sigma k_p^2 (prod_b w_b) u_p

with ``w_a = 1/2`` on the two end nodes of axis a (else 1) and ``e_a = 1`` on
them (else 0). The Helmholtz matrix is ``H = A_{1 - j alpha}`` (Eq. 2); the
shifted-Laplace preconditioner of Eq. 6 is ``M = A_{beta1 - j beta2}``
(the shift enters as ``-(beta1 - j beta2) k^2``; with ``beta = (1, alpha)``
``M`` equals ``H`` and with ``beta = 0`` the interior rows are ``-Lap_h``).
The absorbing term uses the unshifted real ``k`` in both operators.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def axis_weights(n: int):
    """Row weight ``w`` and boundary flag ``e`` along one axis of ``n`` nodes."""
    w = np.ones(n, dtype=np.float64)
    e = np.zeros(n, dtype=np.float64)
    w[0] = w[-1] = 0.5
    e[0] = e[-1] = 1.0
    return w, e


def _along(v: np.ndarray, axis: int, ndim: int) -> np.ndarray:
    """Reshape a 1D per-axis array so that it broadcasts along ``axis``."""
    shape = [1] * ndim
    shape[axis] = -1
    return v.reshape(shape)


def row_weights(shape) -> np.ndarray:
    """Diagonal of ``W`` (product of the per-axis row weights), grid-shaped."""
    ndim = len(shape)
    wt = np.ones(shape, dtype=np.float64)
    for a, n in enumerate(shape):
        wt = wt * _along(axis_weights(n)[0], a, ndim)
    return wt


def _spacing(h, ndim):
    if np.isscalar(h):
        return (float(h),) * ndim
    h = tuple(float(x) for x in h)
    assert len(h) == ndim
    return h


def assemble(m: np.ndarray, omega: float, sigma: complex, h) -> sp.csr_matrix:
    """Sparse ``A_sigma`` for slowness ``m`` (1D or 2D array) and spacing ``h``.

    ``h`` is a scalar or one spacing per axis in storage order
    (``(h_z, h_x)`` in 2D). Returns an ``N x N`` complex128 CSR matrix acting on
    the row-major flattening of the grid.
    """
    m = np.asarray(m, dtype=np.float64)
    shape = m.shape
    ndim = m.ndim
    assert ndim in (1, 2)
    hs = _spacing(h, ndim)
    N = m.size
    k = omega * m
    k2 = k * k
    idx = np.arange(N).reshape(shape)
    weights = [axis_weights(n) for n in shape]

    diag = np.zeros(shape, dtype=np.complex128)
    rows, cols, vals = [], [], []
    for a in range(ndim):
        n_a = shape[a]
        # product of the other axes' row weights
        other = np.ones(shape, dtype=np.float64)
        for b in range(ndim):
            if b != a:
                other = other * _along(weights[b][0], b, ndim)
        coef = other / hs[a] ** 2
        # couplings between node i and node i+1 along axis a
        lo = np.take(idx, np.arange(0, n_a - 1), axis=a).ravel()
        hi = np.take(idx, np.arange(1, n_a), axis=a).ravel()
        c = np.take(coef, np.arange(0, n_a - 1), axis=a).ravel()
        rows += [lo, hi]
        cols += [hi, lo]
        vals += [-c, -c]
        # each neighbour along a contributes +coef to the diagonal
        nnb = np.full(n_a, 2.0)
        nnb[0] = nnb[-1] = 1.0
        diag += coef * _along(nnb, a, ndim)
        # absorbing boundary term of the faces normal to axis a
        diag += 1j * k * _along(weights[a][1], a, ndim) * other / hs[a]
    diag -= sigma * k2 * row_weights(shape)

    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N), dtype=np.complex128)
    return A.tocsr()


def helmholtz(m, omega, alpha, h) -> sp.csr_matrix:
    """``H`` of Eq. 2-3: ``A_sigma`` with ``sigma = 1 - j alpha``."""
    return assemble(m, omega, 1.0 - 1j * alpha, h)


def shifted_laplace(m, omega, beta1, beta2, h) -> sp.csr_matrix:
    """Shifted-Laplace ``M`` of Eq. 6, read as ``-Lap - (beta1 - j beta2) k^2``."""
    return assemble(m, omega, beta1 - 1j * beta2, h)


def weighted_rhs(f: np.ndarray) -> np.ndarray:
    """``b = W f`` (flattened), the right-hand side that goes with ``A_sigma``."""
    f = np.asarray(f, dtype=np.complex128)
    return (row_weights(f.shape) * f).ravel()
