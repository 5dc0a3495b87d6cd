"""Textbook right-preconditioned restarted (flexible) GMRES (oracle; test
infrastructure only).

The paper solves the right-preconditioned system ``H P^{-1} z = f``,
``z = P u`` (Eq. 5-7 with ``M_l = I``, ``M_r = P``) by GMRES (Saad and
Schultz, cited in the Introduction). Restart length, tolerance and initial
guess are not printed in the paper; they are arguments here.

Algorithm (one restart cycle of length ``m``), with the Hermitian product
``<a, b> = sum conj(a_i) b_i``:

1. ``r = b - A x``; stop (converged) if ``||r|| / ||b|| <= tol``;
   ``v_1 = r / ||r||``, ``g = ||r|| e_1``.
2. for ``j = 1..m``: ``z_j = Prec(v_j)``; ``w = A z_j``; modified
   Gram-Schmidt against ``v_1..v_j`` gives ``h_{ij}``; ``h_{j+1,j} = ||w||``.
   Apply the previous Givens rotations to column ``j``, then a new rotation
   that zeroes ``h_{j+1,j}``: with ``a = h_jj``, ``b = h_{j+1,j} >= 0``,
   ``t = sqrt(|a|^2 + b^2)``, ``c = |a|/t``, ``s = (a/|a|) b / t``
   (``c=1, s=0`` if ``b=0``; ``c=0, s=1`` if ``a=0``), acting as
   ``(p, q) -> (c p + s q, -conj(s) p + c q)``. Then
   ``(g_j, g_{j+1}) = (c g_j, -conj(s) g_j)`` and ``|g_{j+1}|/||b||`` is the
   residual estimate. Stop the cycle on a happy breakdown (``h_{j+1,j} = 0``),
   when the estimate is ``<= tol``, or when the iteration budget is spent;
   otherwise ``v_{j+1} = w / h_{j+1,j}``.
3. back-substitute ``R y = g_{1:j}``; flexible: ``x += Z y``; standard:
   ``x += Prec(V y)``. Go to 1. Convergence is declared only on the
   recomputed true residual of step 1.

The unknown ``x`` is the preconditioned-system solution mapped back, i.e. the
wavefield ``u`` itself (``u = P^{-1} z``).
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np

OK = 0
NOT_CONVERGED = 1


@dataclasses.dataclass
class GmresResult:
    x: np.ndarray
    iterations: int
    history: List[float]         # history[0] = 1, history[k] = estimate after step k
    true_rel_res: float
    status: int
    last_cycle: Optional[dict] = None   # V, Z, Hbar of the final cycle (for checks)


def givens(a: complex, b: float):
    """Rotation ``(c, s)`` that maps ``(a, b)`` to ``(t a/|a|, 0)``; ``b >= 0`` real."""
    if b == 0.0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, 1.0 + 0.0j
    t = np.sqrt(abs(a) ** 2 + b * b)
    return abs(a) / t, (a / abs(a)) * (b / t)


def gmres(apply_A: Callable, b: np.ndarray, tol: float, restart: int, maxiter: int,
          prec: Optional[Callable] = None, flexible: bool = True,
          keep_basis: bool = False) -> GmresResult:
    b = np.asarray(b, dtype=np.complex128)
    N = b.size
    if prec is None:
        prec = lambda v: v  # noqa: E731
    beta0 = np.linalg.norm(b)
    x = np.zeros(N, dtype=np.complex128)
    hist = [1.0]
    if beta0 == 0.0:
        return GmresResult(x, 0, hist, 0.0, OK)
    it = 0
    last = None
    while True:
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        rel = beta / beta0
        if not np.isfinite(rel):
            raise FloatingPointError("non-finite residual")
        if rel <= tol:
            return GmresResult(x, it, hist, rel, OK, last)
        if it >= maxiter:
            return GmresResult(x, it, hist, rel, NOT_CONVERGED, last)
        m = restart
        V = np.zeros((m + 1, N), dtype=np.complex128)
        Z = np.zeros((m, N), dtype=np.complex128) if flexible else None
        Hbar = np.zeros((m + 1, m), dtype=np.complex128)   # unrotated, for checks
        Rm = np.zeros((m + 1, m), dtype=np.complex128)     # rotated
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            z = prec(V[j])
            if flexible:
                Z[j] = z
            w = apply_A(z)
            it += 1
            for i in range(j + 1):                      # modified Gram-Schmidt
                hij = np.vdot(V[i], w)
                Hbar[i, j] = hij
                w = w - hij * V[i]
            hn = np.linalg.norm(w)
            Hbar[j + 1, j] = hn
            col = Hbar[: j + 2, j].copy()
            for i in range(j):                          # previous rotations
                p, q = col[i], col[i + 1]
                col[i] = cs[i] * p + sn[i] * q
                col[i + 1] = -np.conj(sn[i]) * p + cs[i] * q
            c, s = givens(col[j], hn)
            cs[j], sn[j] = c, s
            col[j] = c * col[j] + s * col[j + 1]
            col[j + 1] = 0.0
            Rm[: j + 2, j] = col
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            est = abs(g[j + 1]) / beta0
            hist.append(est)
            k = j + 1
            if hn > 0.0:
                V[j + 1] = w / hn
            if hn == 0.0 or est <= tol or it >= maxiter:
                break
        # back substitution R y = g
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - Rm[i, i + 1:k] @ y[i + 1:k]) / Rm[i, i]
        if flexible:
            x = x + Z[:k].T @ y
        else:
            x = x + prec(V[:k].T @ y)
        if keep_basis:
            last = dict(V=V[: k + 1].copy(), Z=(Z[:k].copy() if flexible else None),
                        Hbar=Hbar[: k + 1, :k].copy(), k=k)
