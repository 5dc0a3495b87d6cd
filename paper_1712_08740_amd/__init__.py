"""MI355X-native shifted-Laplace preconditioned GMRES for the heterogeneous
Helmholtz equation (Kazemi, arXiv:1712.08740).

The solver lives in the HIP library ``libhh.so`` (C ABI, ``include/helmholtz.h``);
``paper_1712_08740_amd.hh`` is its thin ctypes binding. PyTorch supplies device
memory and streams only.
"""
__all__ = ["hh"]
