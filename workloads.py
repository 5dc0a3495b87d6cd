"""Seeded synthetic inputs: velocity/slowness models, point sources and the
benchmark workloads.

This module holds input data only. It contains none of the solver's
arithmetic (no operator, no boundary weights, no preconditioner), so both the
CPU oracle tests and the GPU path may take their inputs from it.

Conventions
-----------
* 1D grids have ``n`` nodes at depth ``z_i = i*h``.
* 2D grids are stored ``(nz, nx)`` row-major (x fastest); node ``(iz, ix)``
  sits at ``x = ix*h, z = iz*h``. A grid named "401x201" has nx=401, nz=201.
* The model is returned as slowness ``m = 1/c`` (s/m), float64, C-contiguous.
* A unit point source is ``f[s] = 1`` (complex128), zero elsewhere.

The paper's own models (a 1D well log and the middle of the Marmousi model,
Section "Example") are not printed in it; the layered 1D model and the
Gaussian random-field models below stand in for them with the shapes, spacing
and velocity range of those workloads.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np


# ----------------------------------------------------------------------------
# 1D layered model
# ----------------------------------------------------------------------------
def layered_velocity_1d(n: int = 1001, h: float = 5.0,
                        interfaces=(1500.0, 3500.0),
                        velocities=(1500.0, 2200.0, 3000.0)) -> np.ndarray:
    """Piecewise-constant velocity on ``z_i = i*h``.

    Layers are half-open: layer 0 for ``z < interfaces[0]``, layer 1 for
    ``interfaces[0] <= z < interfaces[1]``, and so on.
    """
    z = np.arange(n, dtype=np.float64) * h
    c = np.full(n, velocities[0], dtype=np.float64)
    for zi, ci in zip(interfaces, velocities[1:]):
        c[z >= zi] = ci
    return c


def homogeneous_velocity(shape, c: float) -> np.ndarray:
    return np.full(shape, float(c), dtype=np.float64)


# ----------------------------------------------------------------------------
# 2D Gaussian random-field model
# ----------------------------------------------------------------------------
def random_field_velocity_2d(nz: int, nx: int, h: float, seed: int,
                             corr_len: float = 200.0,
                             cmin: float = 1500.0, cmax: float = 4500.0) -> np.ndarray:
    """Seeded Gaussian random field with a linear depth gradient.

    White noise (``numpy.random.default_rng(seed)``) is smoothed by a Gaussian
    kernel of standard deviation ``corr_len/(2h)`` grid points, which gives a
    covariance close to ``exp(-r^2/corr_len^2)``. The field is min-max
    normalised to ``g`` in [0, 1] and mapped to
    ``c = cmin + (cmax-cmin) * (g/2 + z/(2 z_max))``.
    """
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((nz, nx))
    g = gaussian_filter(noise, sigma=corr_len / (2.0 * h), mode="reflect")
    g = (g - g.min()) / (g.max() - g.min())
    z = np.arange(nz, dtype=np.float64)[:, None] * h
    zmax = (nz - 1) * h
    c = cmin + (cmax - cmin) * (0.5 * g + 0.5 * z / zmax)
    return np.ascontiguousarray(c, dtype=np.float64)


def point_source(shape, index) -> np.ndarray:
    """Unit point source: ``f[index] = 1``; ``index`` is ``i`` (1D) or ``(iz, ix)``."""
    f = np.zeros(shape, dtype=np.complex128)
    f[index] = 1.0
    return f


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    slowness: np.ndarray          # m = 1/c, float64, shape (n,) or (nz, nx)
    h: float                      # grid spacing (m), equal in x and z
    freq_hz: float
    alpha: float
    source: np.ndarray            # complex128, same shape as slowness
    beta: Tuple[float, float]
    restart: int
    tol: float
    precond: str                  # "exact" (1D tridiagonal) or "mg" (V-cycle)

    @property
    def omega(self) -> float:
        return 2.0 * np.pi * self.freq_hz

    @property
    def shape(self):
        return self.slowness.shape


def layered_1d(n: int = 1001, h: float = 5.0, freq_hz: float = 10.0,
               alpha: float = 0.01, src: int = 100,
               beta=(1.0, 0.5), restart: int = 50, tol: float = 1e-6) -> Workload:
    """1D well: 3 layers of 1500/2200/3000 m/s with tops at 0/1.5/3.5 km."""
    c = layered_velocity_1d(n, h)
    return Workload(name=f"layered1d_n{n}_f{freq_hz:g}", slowness=1.0 / c, h=h,
                    freq_hz=freq_hz, alpha=alpha, source=point_source((n,), src),
                    beta=tuple(beta), restart=restart, tol=tol, precond="exact")


def random_field_2d(nx: int = 401, nz: int = 201, h: float = 10.0, seed: int = 2,
                    freq_hz: float = 10.0, alpha: float = 0.01,
                    src: Optional[Tuple[int, int]] = None,
                    beta=(1.0, 0.5), restart: int = 30, tol: float = 1e-6) -> Workload:
    """2D random-field model; ``src`` is ``(ix, iz)`` (default ``(nx//2, 5)``)."""
    c = random_field_velocity_2d(nz, nx, h, seed)
    if src is None:
        src = (nx // 2, min(5, nz - 1))
    ix, iz = src
    return Workload(name=f"grf2d_{nx}x{nz}_s{seed}_f{freq_hz:g}", slowness=1.0 / c,
                    h=h, freq_hz=freq_hz, alpha=alpha,
                    source=point_source((nz, nx), (iz, ix)), beta=tuple(beta),
                    restart=restart, tol=tol, precond="mg")


def layered_1d_well() -> Workload:
    """n=1001, h=5 m, 10 Hz, alpha=0.01, source at index 100, GMRES(50)."""
    return layered_1d()


def grf_401x201() -> Workload:
    """401x201 (nx x nz), h=10 m, seed 2, 10 Hz, source (ix,iz)=(200,5), FGMRES(30)."""
    return random_field_2d(401, 201, 10.0, seed=2, freq_hz=10.0, src=(200, 5), restart=30)


def grf_1201x401() -> Workload:
    """1201x401, h=10 m, seed 3, 15 Hz, source (600,5), FGMRES(40), tol 1e-8."""
    return random_field_2d(1201, 401, 10.0, seed=3, freq_hz=15.0, src=(600, 5),
                           restart=40, tol=1e-8)


def grf_801x301_sources() -> Tuple[np.ndarray, List[Tuple[int, int]], List[float]]:
    """801x301, seed 4: slowness, 32 top-row sources (ix, iz=0), 4 frequencies."""
    c = random_field_velocity_2d(301, 801, 10.0, seed=4)
    sources = [(12 + 25 * k, 0) for k in range(32)]
    freqs = [5.0, 7.5, 10.0, 12.5]
    return 1.0 / c, sources, freqs


SERVING_GRIDS = [(201, 101), (401, 201), (801, 401), (1601, 601)]   # (nx, nz)


def serving_stream(n_requests: int = 2000, rate_hz: float = 200.0, seed: int = 5):
    """Poisson request stream: arrival time, grid, frequency, per-request model seed."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    t = np.cumsum(gaps)
    grids = rng.integers(0, len(SERVING_GRIDS), size=n_requests)
    freqs = rng.uniform(3.0, 20.0, size=n_requests)
    out = []
    for i in range(n_requests):
        nx, nz = SERVING_GRIDS[int(grids[i])]
        out.append(dict(id=i, t_arrival=float(t[i]), nx=nx, nz=nz,
                        freq_hz=float(freqs[i]), seed=1000 + i, src=(nx // 2, 5)))
    return out


def random_complex(shape, seed: int) -> np.ndarray:
    """Seeded complex128 test vector with standard normal parts."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def smooth_slowness_2d(nz: int, nx: int, h: float, seed: int = 0) -> np.ndarray:
    """Small heterogeneous 2D model for tiny test grids (1500-3000 m/s)."""
    rng = np.random.default_rng(seed)
    c = 1500.0 + 1500.0 * rng.random((nz, nx))
    return np.ascontiguousarray(1.0 / c)
