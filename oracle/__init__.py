"""CPU FP64 oracle for shifted-Laplace preconditioned GMRES on the
constant-density Helmholtz equation (Kazemi, "Application of shifted-Laplace
preconditioners for heterogenous Helmholtz equation -- part 1: Data
modelling", arXiv:1712.08740).

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package. The GPU library never calls it and
shares no code with it: no kernels, headers, helpers, tables or constants.

Plain, slow and written to be read against the paper:

* ``operator``  -- the discrete operator ``A_sigma`` of Eq. 2-3 with the
  first-order absorbing boundary (Section "Data modelling"); ``H`` and the
  shifted Laplacian ``M`` of Eq. 6 are two shifts of it.
* ``direct``    -- the LU solve of Eq. 4 (SciPy SuperLU).
* ``multigrid`` -- one V(2,2) omega-Jacobi cycle on ``M`` as the approximate
  ``M^{-1}`` in 2D.
* ``gmres``     -- textbook right-preconditioned (flexible) GMRES with modified
  Gram-Schmidt and Givens rotations, Eq. 7.
* ``solver``    -- the whole solve: ``H M^{-1} z = W f``, ``u = M^{-1} z``.
* ``spectrum``  -- dense eigenvalues of ``H`` and ``M^{-1} H`` (Fig. 2).

Every function is pinned by a ``-m "not gpu"`` test against something other
than itself (dense LU, closed-form lattice and continuous Green's functions,
manufactured solutions, SciPy's GMRES, eigenvalue bounds). No function here is
"parity unpinned".
"""
from . import operator, direct, multigrid, gmres, solver, spectrum  # noqa: F401
