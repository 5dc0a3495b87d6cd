"""The C-ABI library loads and exports every entry point that
include/helmholtz.h declares; host-side argument checks that run before any
device work. CPU only (no kernel is launched)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "helmholtz.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hh_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1712_08740_amd import hh
    return hh


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib._lib, n), n
    assert sorted(lib.EXPORTED) == names


def test_constants_match_header(lib):
    src = open(HEADER).read()
    for name in ("HH_MAX_COARSE", "HH_MAX_1D", "HH_NO_PRECOND", "HH_PRECOND_F32", "HH_INITIAL_GUESS"):
        v = int(re.search(rf"#define {name} (\d+)", src).group(1))
        assert getattr(lib, name) == v
    for name, val in re.findall(r"(HH_[A-Z_]+)\s*=\s*(-?\d+)", src):
        assert getattr(lib, name) == int(val), name


def test_status_strings(lib):
    for st in (0, 1, -1, -2, -3, -4, -5, 99):
        assert isinstance(lib.status_string(st), str) and lib.status_string(st)


def test_create_rejects_bad_arguments_before_device_work(lib):
    L = lib._lib
    out = ctypes.c_void_p()
    shape = (ctypes.c_int64 * 2)(9, 11)
    fake = ctypes.c_void_p(0x1000)     # never dereferenced: validation fails first
    assert L.hh_create_problem(fake, 3, shape, 60.0, 0.01, 10.0, None, ctypes.byref(out)) == -1
    assert L.hh_create_problem(None, 2, shape, 60.0, 0.01, 10.0, None, ctypes.byref(out)) == -1
    assert L.hh_create_problem(fake, 2, shape, -1.0, 0.01, 10.0, None, ctypes.byref(out)) == -1
    assert L.hh_create_problem(fake, 2, shape, 60.0, -0.1, 10.0, None, ctypes.byref(out)) == -1
    assert L.hh_create_problem(fake, 2, shape, 60.0, 0.01, 0.0, None, ctypes.byref(out)) == -1
    small = (ctypes.c_int64 * 2)(2, 11)
    assert L.hh_create_problem(fake, 2, small, 60.0, 0.01, 10.0, None, ctypes.byref(out)) == -1
    big1d = (ctypes.c_int64 * 2)(lib.HH_MAX_1D + 1, 0)
    assert L.hh_create_problem(fake, 1, big1d, 60.0, 0.01, 10.0, None, ctypes.byref(out)) == -5
    assert "1D" in L.hh_last_error().decode()
    assert out.value is None


def test_null_handles_rejected(lib):
    L = lib._lib
    n = ctypes.c_size_t()
    assert L.hh_workspace_bytes(None, 30, ctypes.byref(n)) == -1
    assert L.hh_set_shift(None, 1.0, 0.5) == -1
    assert L.hh_destroy_problem(None) == 0
    assert L.hh_orthogonalize_scratch_bytes(1000, 0, ctypes.byref(n)) == -1
    assert L.hh_orthogonalize_scratch_bytes(1000, 4, ctypes.byref(n)) == 0 and n.value > 0


def test_footprint_plans_the_oracle_hierarchy(lib):
    """hh_footprint_bytes plans on the host (no device): the operator bytes are
    those of the levels the oracle's coarsening rule gives (9 complex
    coefficients per coarse node and an omega/diag per smoothing node, each in
    complex128 and complex64, m^2 in float64 and float32, the coarsest inverse
    in both precisions and the banded LU of the coarsest stencil), within the
    256-byte alignment of each buffer and the fixed scratch; the workspace
    grows with restart and sources."""
    import numpy as np
    import workloads as wl
    from oracle import multigrid as mg
    cases = [(wl.grf_401x201(), 4096), (wl.grf_401x201(), 1000)]
    slow, _, freqs = wl.grf_801x301_sources()
    for fz in freqs:
        w = wl.random_field_2d(801, 301, 10.0, seed=4, freq_hz=fz, src=(12, 0))
        cases.append((w, 16384))
    for w, mc in cases:
        kmax = w.omega * w.slowness.max()
        shapes = mg.level_shapes(w.shape, (w.h, w.h), kmax, max_coarse=mc)
        n = [a * b for a, b in shapes]
        nc = n[-1]
        bw = min(shapes[-1]) + 1                    # half-bandwidth of the coarsest stencil
        expect = (12 * n[0] + sum(216 * v for v in n[1:]) + sum(24 * v for v in n[:-1])
                  + 24 * nc * nc + 16 * nc * (4 * bw + 2) + 16 * 4096)
        pb, wb = lib.footprint_bytes(w.shape, w.omega, w.slowness.max(), w.h, max_coarse=mc)
        assert expect <= pb <= expect + 256 * (2 * len(n) + 16), (w.name, mc)
        _, wb2 = lib.footprint_bytes(w.shape, w.omega, w.slowness.max(), w.h, max_coarse=mc,
                                     restart=60)
        _, wb3 = lib.footprint_bytes(w.shape, w.omega, w.slowness.max(), w.h, max_coarse=mc,
                                     nrhs=3)
        N = w.slowness.size
        assert wb2 - wb >= 2 * 30 * N * 16          # 30 more V and Z columns
        assert wb3 >= 3 * wb
    # 1D: m^2 in both precisions, the fixed scratch, and the cyclic-reduction
    # multipliers of M (two per step, ten steps for 1001 nodes, plus the final
    # diagonal) in complex128 and complex64
    pb, wb = lib.footprint_bytes((1001,), 2 * np.pi * 10, 1 / 1500, 5.0, restart=50)
    e = (2 * 10 + 1) * 1001
    expect = 12 * 1001 + 16 * 4096 + 24 * e
    assert expect <= pb <= expect + 256 * 8
    assert wb >= (51 + 50) * 1001 * 16


def test_footprint_rejects_bad_arguments(lib):
    with pytest.raises(lib.HHError):
        lib.footprint_bytes((201, 401), -1.0, 1e-3, 10.0)
    with pytest.raises(lib.HHError):
        lib.footprint_bytes((201, 401), 60.0, 1e-3, 10.0, max_coarse=0)
    with pytest.raises(lib.HHError):           # 26 x 26 cannot be coarsened below 100 nodes
        lib.footprint_bytes((201, 401), 60.0, 1 / 1500, 10.0, max_coarse=100)
