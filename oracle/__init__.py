"""Python access to the serial CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are its only users.  It imports nothing from the
HIP package and the HIP package imports nothing from it.

See xs_oracle.h for the definition it computes and the readings of the
paper (section 5.1, the hash-bin paragraph after Table 1) it takes.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

from .build import LIB, build

N_CHANNELS = 5

_lib = None
_libs = {}


class _Tables(ctypes.Structure):
    _fields_ = [
        ("n_nuclides", ctypes.c_int32),
        ("grid_offsets", ctypes.c_void_p),
        ("energy", ctypes.c_void_p),
        ("xs", ctypes.c_void_p),
        ("n_materials", ctypes.c_int32),
        ("mat_offsets", ctypes.c_void_p),
        ("mat_nuclides", ctypes.c_void_p),
        ("mat_density", ctypes.c_void_p),
    ]


def load(path: str = None):
    """Load liboracle.so (building it first if absent), or another build of
    the same source at `path` (the tests load deliberately broken copies to
    show that the pins catch them)."""
    global _lib
    if path is not None:
        if path not in _libs:
            _libs[path] = _declare(ctypes.CDLL(path))
        return _libs[path]
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = _declare(ctypes.CDLL(LIB))
    return _lib


def _declare(lib):
    i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    lib.xso_bracket_count.argtypes = [vp, i64, ctypes.c_double]
    lib.xso_bracket_count.restype = i64
    lib.xso_bracket_bisect.argtypes = [vp, i64, ctypes.c_double]
    lib.xso_bracket_bisect.restype = i64
    lib.xso_lookup.argtypes = [ctypes.POINTER(_Tables), ctypes.c_double,
                               i32, ctypes.c_int, vp, vp]
    lib.xso_lookup.restype = ctypes.c_int
    lib.xso_lookup_batch.argtypes = [ctypes.POINTER(_Tables), i64, vp, vp,
                                     ctypes.c_int, vp, vp, vp]
    lib.xso_lookup_batch.restype = i64
    lib.xso_lookup_batch_f32.argtypes = [ctypes.POINTER(_Tables), i64, vp,
                                         vp, vp]
    lib.xso_lookup_batch_f32.restype = i64
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleTables:
    """Holds contiguous copies of a table set and the C view of them."""

    def __init__(self, t):
        self.grid_offsets = np.ascontiguousarray(t.grid_offsets, dtype=np.int64)
        self.energy = np.ascontiguousarray(t.energy, dtype=np.float64)
        self.xs = np.ascontiguousarray(t.xs, dtype=np.float64).reshape(-1)
        self.mat_offsets = np.ascontiguousarray(t.mat_offsets, dtype=np.int32)
        self.mat_nuclides = np.ascontiguousarray(t.mat_nuclides, dtype=np.int32)
        self.mat_density = np.ascontiguousarray(t.mat_density, dtype=np.float64)
        self.c = _Tables(len(self.grid_offsets) - 1, _ptr(self.grid_offsets).value,
                         _ptr(self.energy).value, _ptr(self.xs).value,
                         len(self.mat_offsets) - 1, _ptr(self.mat_offsets).value,
                         _ptr(self.mat_nuclides).value, _ptr(self.mat_density).value)

    def sizes(self) -> np.ndarray:
        return np.diff(self.mat_offsets).astype(np.int64)


def _as_ot(t) -> OracleTables:
    return t if isinstance(t, OracleTables) else OracleTables(t)


def bracket_count(grid, e: float, lib=None) -> int:
    g = np.ascontiguousarray(grid, dtype=np.float64)
    return int((lib or load()).xso_bracket_count(_ptr(g), len(g), float(e)))


def bracket_bisect(grid, e: float, lib=None) -> int:
    g = np.ascontiguousarray(grid, dtype=np.float64)
    return int((lib or load()).xso_bracket_bisect(_ptr(g), len(g), float(e)))


def index_offsets(t, mat: np.ndarray) -> np.ndarray:
    """[n+1] prefix sum of the material sizes of the queries (0 if invalid)."""
    ot = _as_ot(t)
    sizes = ot.sizes()
    m = np.asarray(mat, dtype=np.int64)
    ok = (m >= 0) & (m < len(sizes))
    L = np.where(ok, sizes[np.clip(m, 0, len(sizes) - 1)], 0)
    off = np.zeros(len(m) + 1, dtype=np.int64)
    off[1:] = np.cumsum(L)
    return off


def lookup(t, E, mat, search: str = "bisect", with_index: bool = False,
           threads: int = 1, lib=None):
    """FP64 lookups in input order.

    Returns out [n, 5] float64, or (out, idx, idx_offsets) with with_index.
    `search` is "bisect" or "count" (the definition, O(n_k) per nuclide).
    `threads` > 1 runs the unmodified serial routine on contiguous slices in
    that many threads (ctypes releases the GIL during the call).
    """
    lib = lib or load()
    ot = _as_ot(t)
    E = np.ascontiguousarray(E, dtype=np.float64)
    mat = np.ascontiguousarray(mat, dtype=np.int32)
    n = len(E)
    out = np.empty((n, N_CHANNELS), dtype=np.float64)
    s = 1 if search == "count" else 0
    if with_index:
        off = index_offsets(ot, mat)
        idx = np.empty(int(off[-1]), dtype=np.int32)
    else:
        off = idx = None

    def run(a, b):
        if b <= a:
            return
        lib.xso_lookup_batch(
            ctypes.byref(ot.c), b - a, _ptr(E[a:]), _ptr(mat[a:]), s,
            _ptr(out[a:]),
            _ptr(off[a:]) if with_index else None,
            _ptr(idx) if with_index else None)

    _run_sliced(run, n, threads)
    if with_index:
        return out, idx, off
    return out


def lookup_f32(t, E, mat, threads: int = 1, lib=None) -> np.ndarray:
    """The FP32 form (FP32 channels and densities, FP64 search and fraction,
    Kahan-compensated FP32 sum).  Returns [n, 5] float32."""
    lib = lib or load()
    ot = _as_ot(t)
    E = np.ascontiguousarray(E, dtype=np.float64)
    mat = np.ascontiguousarray(mat, dtype=np.int32)
    n = len(E)
    out = np.empty((n, N_CHANNELS), dtype=np.float32)

    def run(a, b):
        if b > a:
            lib.xso_lookup_batch_f32(ctypes.byref(ot.c), b - a, _ptr(E[a:]),
                                     _ptr(mat[a:]), _ptr(out[a:]))

    _run_sliced(run, n, threads)
    return out


def _run_sliced(run, n: int, threads: int):
    threads = max(1, int(threads))
    if threads == 1 or n < 2 * threads:
        run(0, n)
        return
    bounds = [n * i // threads for i in range(threads + 1)]
    ts = [threading.Thread(target=run, args=(bounds[i], bounds[i + 1]))
          for i in range(threads)]
    for th in ts:
        th.start()
    for th in ts:
        th.join()
