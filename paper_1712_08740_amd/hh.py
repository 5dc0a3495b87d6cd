"""ctypes binding of the C ABI in ``include/helmholtz.h`` (argument marshalling
only: every step of the solve runs in the library's HIP kernels).

Device arrays are PyTorch CUDA (HIP) tensors: slowness ``float64``, fields
``complex128`` (interleaved), grid-shaped ``(n,)`` or ``(nz, nx)``. The library
must be built (``python -m paper_1712_08740_amd.build``); importing this module
without it raises ``ImportError`` -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import dataclasses
import json
import os
import tempfile
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; HH_LIB_PATH points at another build of the same sources
LIB_PATH = os.environ.get("HH_LIB_PATH") or os.path.join(_HERE, "libhh.so")

HH_OK = 0
HH_NOT_CONVERGED = 1
HH_EINVAL = -1
HH_ENOMEM = -2
HH_EDEVICE = -3
HH_ENUMERIC = -4
HH_EUNSUPPORTED = -5
HH_NO_PRECOND = 1
HH_INITIAL_GUESS = 4
HH_PRECOND_F32 = 2
HH_MAX_COARSE = 4096
HH_MAX_COARSE_LIMIT = 32768
HH_MAX_1D = 1024
HH_MAX_BATCH = 1024
HH_TILE_DEFAULT = -1
HH_TILE_DOWN_COUNT = 3
HH_TILE_UP_COUNT = 3
# tile shapes by id: down legs in coarse nodes, up legs in level nodes (x by z);
# "zmarch": the fine level's down leg marching along z (4x4 on other levels)
TILE_DOWN_SHAPES = ("4x4", "8x4", "zmarch")
TILE_UP_SHAPES = ("8x4", "16x8", "32x8")
HH_KERNEL_NONE = 0
HH_KERNEL_APPLY_DOT = 1
HH_KERNEL_AXPY_DOT = 2
HH_KERNEL_AXPY_NORM = 3
HH_KERNEL_VC_DOWN = 4
HH_KERNEL_VC_UP = 5
HH_KERNEL_GEMV = 6
HH_KERNEL_PCR = 7
HH_KERNEL_VC_DOWN_COARSE = 8
HH_KERNEL_VC_UP_COARSE = 9
HH_KERNEL_REDUCE = 10
HH_KERNEL_GIVENS = 11

EXPORTED = [
    "hh_create_problem", "hh_set_shift", "hh_workspace_bytes", "hh_solve",
    "hh_destroy_problem", "hh_status_string", "hh_last_error", "hh_num_levels",
    "hh_level_info", "hh_apply_operator", "hh_apply_level_operator", "hh_apply_precond",
    "hh_apply_precond_f32",
    "hh_orthogonalize_scratch_bytes", "hh_orthogonalize", "hh_kernel_timer_start",
    "hh_kernel_timer_read", "hh_workspace_bytes_batch", "hh_solve_batch", "hh_set_max_coarse",
    "hh_footprint_bytes", "hh_create_problem_ex", "hh_autotune", "hh_get_tiles",
    "hh_set_tiles",
]

KERNEL_IDS = {"none": HH_KERNEL_NONE, "apply_dot": HH_KERNEL_APPLY_DOT,
              "axpy_dot": HH_KERNEL_AXPY_DOT, "axpy_norm": HH_KERNEL_AXPY_NORM,
              "vc_down": HH_KERNEL_VC_DOWN, "vc_up": HH_KERNEL_VC_UP,
              "gemv": HH_KERNEL_GEMV, "pcr": HH_KERNEL_PCR,
              "vc_down_coarse": HH_KERNEL_VC_DOWN_COARSE, "vc_up_coarse": HH_KERNEL_VC_UP_COARSE,
              "reduce": HH_KERNEL_REDUCE, "givens": HH_KERNEL_GIVENS}

_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_size_p = ctypes.POINTER(ctypes.c_size_t)
_c_i64_p = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with "
                          "`python -m paper_1712_08740_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "hh_create_problem": (ctypes.c_int, [_vp, ctypes.c_int, _c_i64_p, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, _vp,
                                             ctypes.POINTER(_vp)]),
        "hh_set_shift": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double]),
        "hh_workspace_bytes": (ctypes.c_int, [_vp, ctypes.c_int, _c_size_p]),
        "hh_solve": (ctypes.c_int, [_vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_uint, _vp, ctypes.c_size_t, _vp, _c_int_p,
                                    _c_double_p, _c_double_p, ctypes.c_int, _c_int_p, _vp]),
        "hh_destroy_problem": (ctypes.c_int, [_vp]),
        "hh_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "hh_last_error": (ctypes.c_char_p, []),
        "hh_num_levels": (ctypes.c_int, [_vp, _c_int_p]),
        "hh_autotune": (ctypes.c_int, [_vp, ctypes.c_uint, ctypes.c_int, _vp, ctypes.c_size_t,
                                       ctypes.c_int, _vp]),
        "hh_get_tiles": (ctypes.c_int, [_vp, ctypes.c_int, _c_int_p, _c_int_p]),
        "hh_set_tiles": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
        "hh_level_info": (ctypes.c_int, [_vp, ctypes.c_int, _c_i64_p, _c_double_p]),
        "hh_apply_operator": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp]),
        "hh_apply_level_operator": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp]),
        "hh_apply_precond": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
        "hh_apply_precond_f32": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
        "hh_orthogonalize_scratch_bytes": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int,
                                                          _c_size_p]),
        "hh_orthogonalize": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_int, _vp, _vp,
                                            ctypes.c_size_t, _c_double_p, _c_double_p, _vp]),
        "hh_kernel_timer_start": (ctypes.c_int, [_vp, ctypes.c_int]),
        "hh_kernel_timer_read": (ctypes.c_int, [_vp, _c_i64_p, _c_double_p, _c_double_p]),
        "hh_workspace_bytes_batch": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _c_size_p]),
        "hh_set_max_coarse": (ctypes.c_int, [_vp, ctypes.c_int]),
        "hh_create_problem_ex": (ctypes.c_int, [_vp, ctypes.c_int, _c_i64_p, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                                _vp, ctypes.POINTER(_vp)]),
        "hh_footprint_bytes": (ctypes.c_int, [ctypes.c_int, _c_i64_p, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_int, ctypes.c_uint,
                                              _c_size_p, _c_size_p]),
        "hh_solve_batch": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_uint, _vp, ctypes.c_size_t,
                                          _vp, _c_int_p, _c_double_p, _c_int_p, _c_double_p,
                                          ctypes.c_int, _vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


_lib = _load()


def tile_cache_key(level_shapes, precond_f32: bool, nrhs: int) -> str:
    """Key of a tile choice in a cache file: the hierarchy's level grids, the
    cycle's precision and the batch size (the quantities the timings depend
    on, for one kind of GPU)."""
    grids = ",".join(f"{nz}x{nx}" for nz, nx in level_shapes)
    return f"{'c64' if precond_f32 else 'c128'}/rhs{int(nrhs)}/{grids}"


def read_tile_cache(path: str) -> dict:
    """Entries of a tile cache file ({} when it does not exist)."""
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        data = json.load(fh)
    if not isinstance(data, dict):
        raise ValueError(f"{path}: not a tile cache")
    return data


def write_tile_cache(path: str, key: str, tiles) -> None:
    """Adds one entry ([[down, up] per level]) to a tile cache file, written to
    a temporary file and renamed over the old one."""
    data = read_tile_cache(path)
    data[key] = [[int(d), int(u)] for d, u in tiles]
    folder = os.path.dirname(os.path.abspath(path))
    fd, tmp = tempfile.mkstemp(dir=folder, suffix=".tmp")
    with os.fdopen(fd, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def footprint_bytes(shape, omega: float, max_slowness: float, h: float,
                    max_coarse: int = None, restart: int = 30, nrhs: int = 1,
                    precond_f32: bool = False):
    """``hh_footprint_bytes``: (problem bytes, workspace bytes) a solve of this
    size will allocate on the device; host-side planning only."""
    shape = tuple(int(v) for v in shape)
    sh = (ctypes.c_int64 * 2)(*(shape + (0,) * (2 - len(shape))))
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.hh_footprint_bytes(len(shape), sh, float(omega), float(max_slowness), float(h),
                                   HH_MAX_COARSE if max_coarse is None else int(max_coarse),
                                   int(restart), int(nrhs),
                                   HH_PRECOND_F32 if precond_f32 else 0, ctypes.byref(pb),
                                   ctypes.byref(wb)), "hh_footprint_bytes")
    return pb.value, wb.value


class HHError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.hh_last_error().decode() or _lib.hh_status_string(status).decode()
        super().__init__(f"{where}: status {status} ({_lib.hh_status_string(status).decode()}): {msg}")


def _check(status: int, where: str) -> int:
    if status < 0:
        raise HHError(status, where)
    return status


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev_tensor(t: torch.Tensor, dtype, shape, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


@dataclasses.dataclass
class BatchResult:
    u: torch.Tensor                  # (nrhs, *shape) complex128
    iterations: np.ndarray           # (nrhs,)
    true_rel_res: np.ndarray         # (nrhs,)
    status: np.ndarray               # (nrhs,) per-source status
    history: Optional[np.ndarray]    # (nrhs, hist_cap) or None
    overall: int


@dataclasses.dataclass
class SolveResult:
    u: torch.Tensor
    iterations: int
    true_rel_res: float
    history: np.ndarray
    status: int

    @property
    def converged(self) -> bool:
        return self.status == HH_OK


class Problem:
    """``hh_create_problem`` + ``hh_set_shift`` for one slowness model and frequency."""

    def __init__(self, m: torch.Tensor, omega: float, alpha: float, h: float,
                 beta=(1.0, 0.5), stream=None, max_coarse: Optional[int] = None):
        if not isinstance(m, torch.Tensor) or not m.is_cuda or m.dtype != torch.float64:
            raise ValueError("m must be a float64 CUDA tensor")
        if m.dim() not in (1, 2):
            raise ValueError("m must be 1D or 2D")
        m = m.contiguous()
        self.shape = tuple(m.shape)
        self.device = m.device
        self.ndim = m.dim()
        self._handle = _vp()
        shape = (ctypes.c_int64 * 2)(*self.shape)
        self._setup_stream = stream if stream is not None else torch.cuda.current_stream()
        mc = HH_MAX_COARSE if max_coarse is None else int(max_coarse)
        _check(_lib.hh_create_problem_ex(_vp(m.data_ptr()), m.dim(), shape, float(omega),
                                         float(alpha), float(h), mc,
                                         _vp(self._setup_stream.cuda_stream),
                                         ctypes.byref(self._handle)), "hh_create_problem_ex")
        self._ws = {}
        if tuple(beta) != (1.0, 0.5):
            self.set_shift(*beta)

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_handle", None) and self._handle.value:
            _lib.hh_destroy_problem(self._handle)
            self._handle = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- set-up -------------------------------------------------------------
    def set_shift(self, beta1: float, beta2: float):
        _check(_lib.hh_set_shift(self._handle, float(beta1), float(beta2)), "hh_set_shift")

    def set_max_coarse(self, max_coarse: int):
        """``hh_set_max_coarse``: dense limit of the coarsest grid (rebuilds the hierarchy)."""
        _check(_lib.hh_set_max_coarse(self._handle, int(max_coarse)), "hh_set_max_coarse")
        self._ws = {}

    def workspace_bytes(self, restart: int) -> int:
        n = ctypes.c_size_t()
        _check(_lib.hh_workspace_bytes(self._handle, int(restart), ctypes.byref(n)),
               "hh_workspace_bytes")
        return n.value

    def workspace(self, restart: int) -> torch.Tensor:
        ws = self._ws.get(restart)
        if ws is None:
            ws = torch.empty(self.workspace_bytes(restart), dtype=torch.uint8, device=self.device)
            self._ws[restart] = ws
        return ws

    def workspace_bytes_batch(self, restart: int, nrhs: int) -> int:
        n = ctypes.c_size_t()
        _check(_lib.hh_workspace_bytes_batch(self._handle, int(restart), int(nrhs),
                                             ctypes.byref(n)), "hh_workspace_bytes_batch")
        return n.value

    def solve_batch(self, F: torch.Tensor, tol: float = 1e-6, restart: int = 30,
                    max_iters: int = 2000, no_precond: bool = False, precond_f32: bool = False,
                    U: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                    stream=None, hist_cap: int = 0,
                    X0: Optional[torch.Tensor] = None) -> BatchResult:
        """``hh_solve_batch``: F is (nrhs, *shape) complex128, one source per row.
        ``X0`` (same shape) are initial guesses (HH_INITIAL_GUESS), copied into U."""
        if F.dim() != len(self.shape) + 1:
            raise ValueError(f"F must have shape (nrhs, {self.shape})")
        nrhs = F.shape[0]
        _dev_tensor(F, torch.complex128, (nrhs,) + tuple(self.shape), "F")
        if U is None:
            U = torch.empty_like(F)
        else:
            _dev_tensor(U, torch.complex128, (nrhs,) + tuple(self.shape), "U")
        if X0 is not None:
            _dev_tensor(X0, torch.complex128, (nrhs,) + tuple(self.shape), "X0")
            if X0.data_ptr() != U.data_ptr():
                U.copy_(X0)
        need = self.workspace_bytes_batch(restart, nrhs)
        ws = workspace if workspace is not None else torch.empty(need, dtype=torch.uint8,
                                                                 device=self.device)
        if ws.numel() * ws.element_size() < need:
            raise ValueError(f"workspace needs {need} bytes")
        its = (ctypes.c_int * nrhs)()
        rel = (ctypes.c_double * nrhs)()
        sts = (ctypes.c_int * nrhs)()
        hist = np.zeros((nrhs, max(hist_cap, 1)), dtype=np.float64)
        flags = (HH_NO_PRECOND if no_precond else 0) | (HH_PRECOND_F32 if precond_f32 else 0)
        flags |= HH_INITIAL_GUESS if X0 is not None else 0
        st = _check(_lib.hh_solve_batch(self._handle, nrhs, _vp(F.data_ptr()), float(tol),
                                        int(restart), int(max_iters), flags, _vp(ws.data_ptr()),
                                        ws.numel() * ws.element_size(), _vp(U.data_ptr()), its,
                                        rel, sts,
                                        hist.ctypes.data_as(_c_double_p) if hist_cap else None,
                                        int(hist_cap), _vp(_stream_ptr(stream))),
                    "hh_solve_batch")
        return BatchResult(u=U, iterations=np.array(its[:]), true_rel_res=np.array(rel[:]),
                           status=np.array(sts[:]), history=hist if hist_cap else None,
                           overall=st)

    @property
    def num_levels(self) -> int:
        n = ctypes.c_int()
        _check(_lib.hh_num_levels(self._handle, ctypes.byref(n)), "hh_num_levels")
        return n.value

    def get_tiles(self, level: int):
        """``(down, up)`` tile shape ids of level ``level``'s legs (-1: default)."""
        d, u = ctypes.c_int(), ctypes.c_int()
        _check(_lib.hh_get_tiles(self._handle, int(level), ctypes.byref(d), ctypes.byref(u)),
               "hh_get_tiles")
        return d.value, u.value

    def set_tiles(self, level: int, down: int, up: int):
        _check(_lib.hh_set_tiles(self._handle, int(level), int(down), int(up)), "hh_set_tiles")

    def autotune(self, precond_f32: bool = False, nrhs: int = 1, cache: Optional[str] = None,
                 reps: int = 10, stream=None):
        """Tile shapes of the multigrid legs chosen by timing (``hh_autotune``),
        for the complex64 or complex128 cycle and batches of ``nrhs`` sources.
        With ``cache`` (a JSON file) a choice stored for the same hierarchy,
        precision and batch size is reused instead of timed, and a new one is
        stored. Returns ``[(down, up)]`` per level with legs."""
        nlegs = self.num_levels - 1 if self.ndim == 2 else 0
        if nlegs < 1:
            return []
        key = tile_cache_key([self.level_info(l)[0] for l in range(self.num_levels)],
                             precond_f32, nrhs)
        if cache is not None:
            hit = read_tile_cache(cache).get(key)
            if hit is not None and len(hit) == nlegs:
                for l, (d, u) in enumerate(hit):
                    self.set_tiles(l, d, u)
                return [tuple(t) for t in hit]
        ws = torch.empty(self.workspace_bytes_batch(1, nrhs), dtype=torch.uint8,
                         device=self.device)
        _check(_lib.hh_autotune(self._handle, HH_PRECOND_F32 if precond_f32 else 0, int(nrhs),
                                _vp(ws.data_ptr()), ws.numel(), int(reps),
                                _vp(_stream_ptr(stream))), "hh_autotune")
        tiles = [self.get_tiles(l) for l in range(nlegs)]
        if cache is not None:
            write_tile_cache(cache, key, tiles)
        return tiles

    def level_info(self, level: int):
        shape = (ctypes.c_int64 * 2)()
        spacing = (ctypes.c_double * 2)()
        _check(_lib.hh_level_info(self._handle, int(level), shape, spacing), "hh_level_info")
        return (int(shape[0]), int(shape[1])), (float(spacing[0]), float(spacing[1]))

    def level_shape(self, level: int):
        (nz, nx), _ = self.level_info(level)
        return (nx,) if self.ndim == 1 else (nz, nx)

    # -- kernel timing ------------------------------------------------------
    def kernel_timer_start(self, kernel: str):
        """Bracket every launch of one kernel class in later solves with HIP events."""
        _check(_lib.hh_kernel_timer_start(self._handle, KERNEL_IDS[kernel]),
               "hh_kernel_timer_start")

    def kernel_timer_read(self):
        """``(launches, total_ms, total_algorithmic_bytes)`` since the last start."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        _check(_lib.hh_kernel_timer_read(self._handle, ctypes.byref(n), ctypes.byref(ms),
                                         ctypes.byref(by)), "hh_kernel_timer_read")
        return n.value, ms.value, by.value

    # -- steps --------------------------------------------------------------
    def apply_operator(self, x: torch.Tensor, which: str = "H", y=None, stream=None):
        _dev_tensor(x, torch.complex128, self.shape, "x")
        y = torch.empty_like(x) if y is None else _dev_tensor(y, torch.complex128, self.shape, "y")
        w = {"H": 0, "M": 1}[which]
        _check(_lib.hh_apply_operator(self._handle, w, _vp(x.data_ptr()), _vp(y.data_ptr()),
                                      _vp(_stream_ptr(stream))), "hh_apply_operator")
        return y

    def apply_level_operator(self, level: int, x: torch.Tensor, stream=None):
        shape = self.level_shape(level)
        _dev_tensor(x, torch.complex128, shape, "x")
        y = torch.empty_like(x)
        _check(_lib.hh_apply_level_operator(self._handle, int(level), _vp(x.data_ptr()),
                                            _vp(y.data_ptr()), _vp(_stream_ptr(stream))),
               "hh_apply_level_operator")
        return y

    def apply_precond(self, v: torch.Tensor, stream=None, f32: bool = False):
        """z = M^{-1} v (complex128), or with ``f32`` the complex64 preconditioner
        (z complex64)."""
        _dev_tensor(v, torch.complex128, self.shape, "v")
        z = torch.empty(v.shape, dtype=torch.complex64 if f32 else torch.complex128,
                        device=v.device)
        ws = self.workspace(1)
        fn = _lib.hh_apply_precond_f32 if f32 else _lib.hh_apply_precond
        _check(fn(self._handle, _vp(v.data_ptr()), _vp(z.data_ptr()), _vp(ws.data_ptr()),
                  ws.numel(), _vp(_stream_ptr(stream))),
               "hh_apply_precond_f32" if f32 else "hh_apply_precond")
        return z

    def solve(self, f: torch.Tensor, tol: float = 1e-6, restart: int = 30,
              max_iters: int = 2000, no_precond: bool = False, u: Optional[torch.Tensor] = None,
              workspace: Optional[torch.Tensor] = None, stream=None,
              hist_cap: Optional[int] = None, precond_f32: bool = False,
              x0: Optional[torch.Tensor] = None) -> SolveResult:
        """Right-preconditioned FGMRES(restart) to ``tol`` (``hh_solve``).
        ``precond_f32`` runs the preconditioner in complex64 (HH_PRECOND_F32).
        ``x0`` is an initial guess (HH_INITIAL_GUESS), copied into ``u``: a solve
        that returned HH_NOT_CONVERGED resumes from its ``u``."""
        _dev_tensor(f, torch.complex128, self.shape, "f")
        if u is None:
            u = torch.empty_like(f)
        else:
            _dev_tensor(u, torch.complex128, self.shape, "u")
        if x0 is not None:
            _dev_tensor(x0, torch.complex128, self.shape, "x0")
            if x0.data_ptr() != u.data_ptr():
                u.copy_(x0)
        ws = workspace if workspace is not None else self.workspace(restart)
        need = self.workspace_bytes(restart)
        if ws.numel() * ws.element_size() < need:
            raise ValueError(f"workspace needs {need} bytes")
        cap = (max_iters + 1) if hist_cap is None else int(hist_cap)
        hist = np.zeros(max(cap, 1), dtype=np.float64)
        its = ctypes.c_int()
        rel = ctypes.c_double()
        hlen = ctypes.c_int()
        flags = (HH_NO_PRECOND if no_precond else 0) | (HH_PRECOND_F32 if precond_f32 else 0)
        flags |= HH_INITIAL_GUESS if x0 is not None else 0
        st = _check(_lib.hh_solve(self._handle, _vp(f.data_ptr()), float(tol), int(restart),
                                  int(max_iters), flags, _vp(ws.data_ptr()),
                                  ws.numel() * ws.element_size(), _vp(u.data_ptr()),
                                  ctypes.byref(its), ctypes.byref(rel),
                                  hist.ctypes.data_as(_c_double_p), cap, ctypes.byref(hlen),
                                  _vp(_stream_ptr(stream))), "hh_solve")
        return SolveResult(u=u, iterations=its.value, true_rel_res=rel.value,
                           history=hist[: min(hlen.value, cap)].copy(), status=st)


def orthogonalize(V: torch.Tensor, w: torch.Tensor, stream=None):
    """CGS2 step (``hh_orthogonalize``): ``V`` is ``(k, n)`` complex128 with
    orthonormal rows, ``w`` ``(n,)`` is orthogonalised in place. Returns
    ``(h, ||w||)`` with ``h`` the ``k`` projection coefficients (numpy)."""
    if V.dim() != 2:
        raise ValueError("V must be (k, n)")
    k, n = V.shape
    _dev_tensor(V, torch.complex128, (k, n), "V")
    _dev_tensor(w, torch.complex128, (n,), "w")
    need = ctypes.c_size_t()
    _check(_lib.hh_orthogonalize_scratch_bytes(n, k, ctypes.byref(need)),
           "hh_orthogonalize_scratch_bytes")
    scratch = torch.empty(need.value, dtype=torch.uint8, device=V.device)
    h = np.zeros(2 * k, dtype=np.float64)
    nrm = ctypes.c_double()
    _check(_lib.hh_orthogonalize(_vp(V.data_ptr()), n, k, _vp(w.data_ptr()),
                                 _vp(scratch.data_ptr()), need.value,
                                 h.ctypes.data_as(_c_double_p), ctypes.byref(nrm),
                                 _vp(_stream_ptr(stream))), "hh_orthogonalize")
    return h.view(np.complex128), nrm.value


def status_string(status: int) -> str:
    return _lib.hh_status_string(int(status)).decode()
