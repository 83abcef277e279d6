"""ctypes binding of libxs.so with the same names as include/xs.h.

Argument marshalling only: every step of a lookup runs in the library's HIP
kernels.  torch supplies device memory (output and workspace tensors) and the
HIP stream (torch.cuda.current_stream()).  If libxs.so has not been built the
first call raises; nothing here falls back to another implementation.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxs.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "xs.h")

XS_OK, XS_EINVAL, XS_ETABLE, XS_ENOTBUILT = 0, -1, -2, -3
XS_EWORKSPACE, XS_ENOMEM, XS_EHIP, XS_ETIMEOUT = -4, -5, -6, -7
XS_AUTO = -1
XS_CHANNELS = 5
XS_GRID_NUCLIDE, XS_GRID_HASH, XS_GRID_UNIONIZED = 0, 1, 2
XS_FP64, XS_FP32 = 0, 1
XS_SORT_NONE, XS_SORT_MATERIAL, XS_SORT_ENERGY, XS_SORT_MATERIAL_ENERGY = 0, 1, 2, 3
XS_SORT_BAND_MATERIAL = 4
XS_QUEUE_COMPACT, XS_QUEUE_PREDICATED = 0, 1
XS_BUILD_FP32, XS_BUILD_HASH, XS_BUILD_UNIONIZED = 1, 2, 4
XS_BUILD_UNION_BY_MATERIAL = 8
XS_BUILD_FP32_PAIRS = 16
XS_MAX_HASH_GRIDS = 8
XS_NOALLOC_SCRATCH_BYTES = 128 << 20
XS_NOALLOC_MAX_SORTED = 8323456
INT64_MAX = (1 << 63) - 1

GRIDS = {"nuclide": XS_GRID_NUCLIDE, "hash": XS_GRID_HASH,
         "unionized": XS_GRID_UNIONIZED}
SORTS = {"none": XS_SORT_NONE, "material": XS_SORT_MATERIAL,
         "energy": XS_SORT_ENERGY, "material_energy": XS_SORT_MATERIAL_ENERGY,
         "band_material": XS_SORT_BAND_MATERIAL}


class XsError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {message} (status {status})")
        self.status = status


class xs_table_desc(ctypes.Structure):
    _fields_ = [
        ("n_nuclides", ctypes.c_int32),
        ("n_channels", ctypes.c_int32),
        ("grid_offsets", ctypes.c_void_p),
        ("energy", ctypes.c_void_p),
        ("xs", ctypes.c_void_p),
        ("n_materials", ctypes.c_int32),
        ("mat_offsets", ctypes.c_void_p),
        ("mat_nuclides", ctypes.c_void_p),
        ("mat_density", ctypes.c_void_p),
        ("build_flags", ctypes.c_uint32),
        ("n_hash_bins", ctypes.c_int32),
        ("n_extra_hash_grids", ctypes.c_int32),
        ("extra_hash_bins", ctypes.c_void_p),
    ]


class xs_params(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("grid", ctypes.c_int32),
        ("sort", ctypes.c_int32),
        ("block_size", ctypes.c_int32),
        ("lookups_per_thread", ctypes.c_int32),
        ("lds_stage", ctypes.c_int32),
        ("sort_threshold", ctypes.c_int64),
        ("queue", ctypes.c_int32),
        ("unroll", ctypes.c_int32),
        ("wave_per_lookup", ctypes.c_int32),
        ("hash_bins", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class xs_table_info_t(ctypes.Structure):
    _fields_ = [
        ("n_nuclides", ctypes.c_int32),
        ("n_materials", ctypes.c_int32),
        ("max_material_size", ctypes.c_int32),
        ("n_hash_bins", ctypes.c_int32),
        ("n_points", ctypes.c_int64),
        ("union_size", ctypes.c_int64),
        ("build_flags", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("e_min", ctypes.c_double),
        ("e_max", ctypes.c_double),
        ("n_hash_grids", ctypes.c_int32),
        ("hash_bins", ctypes.c_int32 * XS_MAX_HASH_GRIDS),
        ("reserved2", ctypes.c_int32),
        ("checksum", ctypes.c_uint64),
        ("bytes_grid", ctypes.c_size_t),
        ("bytes_fp64", ctypes.c_size_t),
        ("bytes_fp32", ctypes.c_size_t),
        ("bytes_materials", ctypes.c_size_t),
        ("bytes_hash", ctypes.c_size_t),
        ("bytes_union", ctypes.c_size_t),
    ]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_
             if f not in ("reserved", "reserved2")}
        d["hash_bins"] = list(self.hash_bins)[:self.n_hash_grids]
        return d


class xs_debug_info(ctypes.Structure):
    _fields_ = [
        ("on", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("calls", ctypes.c_int64),
        ("invalid_queries", ctypes.c_int64),
        ("hash_bin_scans", ctypes.c_int64),
        ("hash_full_searches", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class xs_profile_t(ctypes.Structure):
    _fields_ = [
        ("ms_sort", ctypes.c_double),
        ("ms_lookup", ctypes.c_double),
        ("ms_total", ctypes.c_double),
        ("calls", ctypes.c_int64),
        ("sorted_calls", ctypes.c_int64),
        ("lookups", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class xs_tune_config(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("strategy", ctypes.c_int32),
        ("max_evals", ctypes.c_int32),
        ("init_samples", ctypes.c_int32),
        ("batch", ctypes.c_int32),
        ("reps", ctypes.c_int32),
        ("warmup", ctypes.c_int32),
        ("active", ctypes.c_int32),
        ("timeout_factor", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("grid_mask", ctypes.c_uint32),
        ("sort_mask", ctypes.c_uint32),
        ("n_hash_grids", ctypes.c_int32),
        ("hash_bins", ctypes.c_int32 * XS_MAX_HASH_GRIDS),
        ("confirm", ctypes.c_int32),
    ]


class xs_tune_result(ctypes.Structure):
    _fields_ = [
        ("best", xs_params),
        ("best_ms", ctypes.c_double),
        ("baseline", xs_params),
        ("baseline_ms", ctypes.c_double),
        ("evaluated", ctypes.c_int32),
        ("cut", ctypes.c_int32),
        ("space_size", ctypes.c_int32),
        ("best_eval", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("from_cache", ctypes.c_int32),
        ("measured", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {"best": self.best.as_dict(), "best_ms": self.best_ms,
                "baseline": self.baseline.as_dict(),
                "baseline_ms": self.baseline_ms, "evaluated": self.evaluated,
                "cut": self.cut, "space_size": self.space_size,
                "best_eval": self.best_eval, "n": self.n,
                "from_cache": self.from_cache, "measured": self.measured}


class xs_tune_request(ctypes.Structure):
    _fields_ = [
        ("n_sizes", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("sizes", ctypes.c_void_p),
        ("d_E", ctypes.c_void_p),
        ("d_mat", ctypes.c_void_p),
        ("d_active", ctypes.c_void_p),
        ("d_out", ctypes.c_void_p),
        ("d_ws", ctypes.c_void_p),
        ("ws_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
        ("cache_path", ctypes.c_char_p),
        ("config", xs_tune_config),
    ]


class xs_tune_key(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_char * 96),
        ("checksum", ctypes.c_uint64),
        ("precision", ctypes.c_int32),
        ("active", ctypes.c_int32),
        ("size_class", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class xs_request(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("d_E", ctypes.c_void_p),
        ("d_mat", ctypes.c_void_p),
        ("d_out", ctypes.c_void_p),
    ]


class xs_request_stats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("start_us", ctypes.c_double),
        ("end_us", ctypes.c_double),
        ("latency_us", ctypes.c_double),
    ]


class xs_event_config(ctypes.Structure):
    _fields_ = [
        ("n_slots", ctypes.c_int64),
        ("n_histories", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
        ("e_cut", ctypes.c_double),
        ("check_every", ctypes.c_int32),
        ("max_iterations", ctypes.c_int32),
    ]


class xs_event_buffers(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in (
        "E", "mat", "alive", "hist", "ncoll", "sigma", "counters",
        "t_collisions", "t_energy", "t_fate")]


class xs_event_result(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int64),
        ("lookups", ctypes.c_int64),
        ("histories", ctypes.c_int64),
    ]


XS_TUNE_EXHAUSTIVE, XS_TUNE_FOREST = 0, 1
EVAL_FN = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.POINTER(xs_params),
                           ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                           ctypes.c_void_p)

_lib = None


def declared_functions() -> list:
    """Names of the functions include/xs.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(
        r"^(?:xs_status|const char\*)\s+(xs_[a-z_0-9]+)\s*\(", text, re.M)))


def load_library(path: str = LIB_PATH):
    """Load libxs.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with __graft_entry__.build() or "
            "python paper_2402_09222_amd/build.py")
    try:
        # torch bundles a HIP runtime; loading it first makes libxs.so bind to
        # that same runtime instead of a second copy.
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    i32, i64, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "xs_create_tables": ([P(xs_table_desc), vp, P(vp)], i32),
        "xs_destroy_tables": ([vp], i32),
        "xs_table_info": ([vp, P(xs_table_info_t)], i32),
        "xs_params_default": ([P(xs_params), i32], i32),
        "xs_resolve_params": ([vp, i64, P(xs_params), P(xs_params)], i32),
        "xs_workspace_size": ([vp, i64, P(xs_params), P(sz)], i32),
        "xs_lookup_batch": ([vp, i64, vp, vp, vp, P(xs_params), vp, sz, vp], i32),
        "xs_lookup_batch_noalloc": ([vp, i64, vp, vp, vp, P(xs_params), vp],
                                    i32),
        "xs_lookup_active": ([vp, i64, vp, vp, vp, vp, P(xs_params), vp, sz, vp],
                             i32),
        "xs_lookup_indices": ([vp, i64, vp, vp, vp, vp, i32, vp], i32),
        "xs_profile_begin": ([vp], i32),
        "xs_profile_end": ([vp, P(xs_profile_t)], i32),
        "xs_set_debug": ([vp, i32], i32),
        "xs_debug_counters": ([vp, P(xs_debug_info)], i32),
        "xs_tune_config_default": ([P(xs_tune_config)], i32),
        "xs_tune_search": ([ctypes.c_uint32, P(xs_tune_config), EVAL_FN, vp,
                            P(xs_tune_result)], i32),
        "xs_tune": ([vp, P(xs_tune_request), P(xs_tune_result)], i32),
        "xs_set_tuned": ([vp, i64, i32, P(xs_params)], i32),
        "xs_tune_load": ([vp, ctypes.c_char_p, P(i32)], i32),
        "xs_tune_key_of": ([vp, i32, i32, i64, P(xs_tune_key)], i32),
        "xs_tune_cache_get": ([ctypes.c_char_p, P(xs_tune_key), P(xs_params),
                               P(ctypes.c_double)], i32),
        "xs_tune_cache_put": ([ctypes.c_char_p, P(xs_tune_key), P(xs_params),
                               ctypes.c_double], i32),
        "xs_stream_create": ([vp, P(xs_params), i32, vp, P(vp)], i32),
        "xs_stream_submit": ([vp, P(xs_request), i32], i32),
        "xs_stream_wait": ([vp, P(xs_request_stats), P(ctypes.c_double)], i32),
        "xs_stream_params": ([vp, P(xs_params)], i32),
        "xs_stream_destroy": ([vp], i32),
        "xs_lookup_requests": ([vp, P(xs_request), i32, P(xs_params), vp, sz, vp],
                               i32),
        "xs_requests_workspace_size": ([vp, P(xs_request), i32, P(xs_params),
                                        P(sz)], i32),
        "xs_requests_stats": ([vp, i32, vp, P(xs_request_stats),
                               P(ctypes.c_double)], i32),
        "xs_event_workspace_size": ([vp, P(xs_event_config), P(xs_params),
                                     P(sz)], i32),
        "xs_event_run": ([vp, P(xs_event_config), P(xs_event_buffers),
                          P(xs_params), vp, sz, vp, P(xs_event_result)], i32),
        "xs_status_string": ([i32], ctypes.c_char_p),
        "xs_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != XS_OK:
        lib = load_library()
        msg = lib.xs_last_error().decode() or lib.xs_status_string(status).decode()
        raise XsError(status, where, msg)


def xs_status_string(status: int) -> str:
    return load_library().xs_status_string(status).decode()


def xs_last_error() -> str:
    return load_library().xs_last_error().decode()


def _stream_ptr(stream, device=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def make_params(precision=XS_FP64, grid=XS_AUTO, sort=XS_AUTO, block_size=0,
                lookups_per_thread=0, lds_stage=XS_AUTO, sort_threshold=-1,
                queue=XS_AUTO, unroll=0, wave_per_lookup=XS_AUTO,
                hash_bins=XS_AUTO) -> xs_params:
    if isinstance(grid, str):
        grid = GRIDS[grid]
    if isinstance(sort, str):
        sort = SORTS[sort]
    return xs_params(precision, grid, sort, block_size, lookups_per_thread,
                     lds_stage, sort_threshold, queue, unroll, wave_per_lookup,
                     hash_bins)


class Tables:
    """Owns an xs_tables_t handle (freed by close() or garbage collection)."""

    def __init__(self, handle: ctypes.c_void_p):
        self.handle = handle

    def close(self):
        if self.handle and self.handle.value:
            _check(load_library().xs_destroy_tables(self.handle),
                   "xs_destroy_tables")
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def _as_parameter_(self):
        return self.handle


def make_desc(t, build_flags: int = 0, n_hash_bins: int = 0,
              extra_hash_bins=()):
    """xs_table_desc over host numpy arrays of a table set (any object with
    grid_offsets, energy, xs, mat_offsets, mat_nuclides, mat_density).
    Returns (desc, keep) where keep holds the arrays alive."""
    import numpy as np
    extra = np.ascontiguousarray(list(extra_hash_bins), dtype=np.int32)
    keep = dict(
        extra_hash_bins=extra,
        grid_offsets=np.ascontiguousarray(t.grid_offsets, dtype=np.int64),
        energy=np.ascontiguousarray(t.energy, dtype=np.float64),
        xs=np.ascontiguousarray(t.xs, dtype=np.float64).reshape(-1),
        mat_offsets=np.ascontiguousarray(t.mat_offsets, dtype=np.int32),
        mat_nuclides=np.ascontiguousarray(t.mat_nuclides, dtype=np.int32),
        mat_density=np.ascontiguousarray(t.mat_density, dtype=np.float64),
    )
    d = xs_table_desc(
        len(keep["grid_offsets"]) - 1, XS_CHANNELS,
        keep["grid_offsets"].ctypes.data, keep["energy"].ctypes.data,
        keep["xs"].ctypes.data, len(keep["mat_offsets"]) - 1,
        keep["mat_offsets"].ctypes.data, keep["mat_nuclides"].ctypes.data,
        keep["mat_density"].ctypes.data, build_flags, n_hash_bins,
        len(extra), extra.ctypes.data if len(extra) else None)
    return d, keep


def xs_create_tables(t, build_flags: int = XS_BUILD_FP32 | XS_BUILD_HASH,
                     n_hash_bins: int = 4000, stream=None,
                     extra_hash_bins=()) -> Tables:
    """Upload a table set (see make_desc) and build the requested structures.
    The paper's default bin count is 4,000; extra_hash_bins adds further hash
    grids (the tuner's hash-bin choices)."""
    lib = load_library()
    desc, keep = make_desc(t, build_flags, n_hash_bins, extra_hash_bins)
    h = ctypes.c_void_p()
    s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
    _check(lib.xs_create_tables(ctypes.byref(desc), s, ctypes.byref(h)),
           "xs_create_tables")
    del keep
    return Tables(h)


def xs_destroy_tables(tables: Tables):
    tables.close()


def xs_table_info(tables: Tables) -> dict:
    info = xs_table_info_t()
    _check(load_library().xs_table_info(tables.handle, ctypes.byref(info)),
           "xs_table_info")
    return info.as_dict()


def xs_params_default(precision: int = XS_FP64) -> xs_params:
    p = xs_params()
    _check(load_library().xs_params_default(ctypes.byref(p), precision),
           "xs_params_default")
    return p


def xs_resolve_params(tables: Tables, n: int, params: xs_params = None) -> xs_params:
    out = xs_params()
    _check(load_library().xs_resolve_params(
        tables.handle, n, ctypes.byref(params) if params is not None else None,
        ctypes.byref(out)), "xs_resolve_params")
    return out


def xs_workspace_size(tables: Tables, n: int, params: xs_params = None) -> int:
    b = ctypes.c_size_t()
    _check(load_library().xs_workspace_size(
        tables.handle, n, ctypes.byref(params) if params is not None else None,
        ctypes.byref(b)), "xs_workspace_size")
    return b.value


def _workspace(nbytes: int, device):
    """A 256-byte aligned device buffer of nbytes (torch uint8 tensor, ptr)."""
    import torch
    if nbytes == 0:
        return None, None, 0
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    ptr = buf.data_ptr()
    off = (-ptr) % 256
    return buf, ctypes.c_void_p(ptr + off), nbytes


def _out_tensor(n, params, device, out):
    import torch
    prec = params.precision if params is not None else XS_FP64
    dt = torch.float64 if prec == XS_FP64 else torch.float32
    if out is None:
        return torch.empty((n, XS_CHANNELS), dtype=dt, device=device)
    if out.dtype != dt or out.shape[0] < n or not out.is_contiguous():
        raise ValueError("out must be a contiguous [n, 5] tensor of the "
                         "precision's dtype")
    return out


def _check_queries(E, mat):
    import torch
    if E.dtype != torch.float64 or mat.dtype != torch.int32:
        raise TypeError("E must be float64 and mat int32")
    if not (E.is_cuda and mat.is_cuda):
        raise TypeError("E and mat must be device tensors")
    if not (E.is_contiguous() and mat.is_contiguous()) or E.numel() != mat.numel():
        raise ValueError("E and mat must be contiguous and of equal length")


def xs_lookup_batch(tables: Tables, E, mat, out=None, params: xs_params = None,
                    workspace=None, stream=None):
    """out[q, c] = macroscopic value of channel c for (E[q], mat[q]).
    E: float64 device tensor [n]; mat: int32 device tensor [n].  Returns out
    ([n, 5], float64 for XS_FP64, float32 for XS_FP32)."""
    _check_queries(E, mat)
    n = E.numel()
    out = _out_tensor(n, params, E.device, out)
    pp = ctypes.byref(params) if params is not None else None
    if workspace is None:
        nb = xs_workspace_size(tables, n, params)
        keep, ws, nb = _workspace(nb, E.device)
    else:
        keep, ws, nb = workspace
    _check(load_library().xs_lookup_batch(
        tables.handle, n, ctypes.c_void_p(E.data_ptr()),
        ctypes.c_void_p(mat.data_ptr()), ctypes.c_void_p(out.data_ptr()), pp,
        ws, nb, _stream_ptr(stream, E.device)), "xs_lookup_batch")
    return out


def xs_lookup_batch_noalloc(tables: Tables, E, mat, out=None,
                            params: xs_params = None, stream=None):
    """xs_lookup_batch with the sort's scratch in the library's fixed device
    array (no workspace, no allocation inside the call).  Returns out."""
    _check_queries(E, mat)
    n = E.numel()
    out = _out_tensor(n, params, E.device, out)
    pp = ctypes.byref(params) if params is not None else None
    _check(load_library().xs_lookup_batch_noalloc(
        tables.handle, n, ctypes.c_void_p(E.data_ptr()),
        ctypes.c_void_p(mat.data_ptr()), ctypes.c_void_p(out.data_ptr()), pp,
        _stream_ptr(stream, E.device)), "xs_lookup_batch_noalloc")
    return out


def xs_lookup_active(tables: Tables, E, mat, active, out, params: xs_params = None,
                     workspace=None, stream=None):
    """As xs_lookup_batch for slots with active[q] != 0 (uint8 device
    tensor); other rows of `out` are left as they were."""
    import torch
    _check_queries(E, mat)
    if active.dtype != torch.uint8 or active.numel() != E.numel():
        raise TypeError("active must be a uint8 tensor of length n")
    n = E.numel()
    out = _out_tensor(n, params, E.device, out)
    pp = ctypes.byref(params) if params is not None else None
    if workspace is None:
        nb = xs_workspace_size(tables, n, params)
        keep, ws, nb = _workspace(nb, E.device)
    else:
        keep, ws, nb = workspace
    _check(load_library().xs_lookup_active(
        tables.handle, n, ctypes.c_void_p(E.data_ptr()),
        ctypes.c_void_p(mat.data_ptr()), ctypes.c_void_p(active.data_ptr()),
        ctypes.c_void_p(out.data_ptr()), pp, ws, nb,
        _stream_ptr(stream, E.device)), "xs_lookup_active")
    return out


def xs_lookup_indices(tables: Tables, E, mat, idx_offsets, grid=XS_GRID_NUCLIDE,
                      idx=None, stream=None):
    """Brackets of every (lookup, nuclide) pair with the given grid method.
    idx_offsets: int64 device tensor [n+1].  Returns idx (int32 [total])."""
    import torch
    _check_queries(E, mat)
    if isinstance(grid, str):
        grid = GRIDS[grid]
    total = int(idx_offsets[-1].item()) if idx_offsets.numel() else 0
    if idx is None:
        idx = torch.full((max(total, 1),), -2, dtype=torch.int32, device=E.device)
    _check(load_library().xs_lookup_indices(
        tables.handle, E.numel(), ctypes.c_void_p(E.data_ptr()),
        ctypes.c_void_p(mat.data_ptr()), ctypes.c_void_p(idx_offsets.data_ptr()),
        ctypes.c_void_p(idx.data_ptr()), grid, _stream_ptr(stream, E.device)),
        "xs_lookup_indices")
    return idx[:total]


def xs_profile_begin(tables: Tables):
    _check(load_library().xs_profile_begin(tables.handle), "xs_profile_begin")


def xs_profile_end(tables: Tables) -> dict:
    p = xs_profile_t()
    _check(load_library().xs_profile_end(tables.handle, ctypes.byref(p)),
           "xs_profile_end")
    return p.as_dict()


def xs_set_debug(tables: Tables, on: bool) -> None:
    _check(load_library().xs_set_debug(tables.handle, 1 if on else 0),
           "xs_set_debug")


def xs_debug_counters(tables: Tables) -> dict:
    d = xs_debug_info()
    _check(load_library().xs_debug_counters(tables.handle, ctypes.byref(d)),
           "xs_debug_counters")
    return d.as_dict()


def xs_tune_config_default(**over) -> xs_tune_config:
    """Default tuner configuration with fields overridden by keyword."""
    c = xs_tune_config()
    _check(load_library().xs_tune_config_default(ctypes.byref(c)),
           "xs_tune_config_default")
    for k, v in over.items():
        if k == "hash_bins":  # a list: the hash grids on offer
            c.n_hash_grids = len(v)
            for i, b in enumerate(v):
                c.hash_bins[i] = b
        else:
            setattr(c, k, v)
    return c


def xs_tune_search(built_grids: int, cfg: xs_tune_config, evaluate) -> xs_tune_result:
    """Run the search with a Python evaluator evaluate(params, cutoff_ms) ->
    milliseconds (no device needed)."""
    err = []

    def cb(p, cutoff, ms, user):
        try:
            ms[0] = float(evaluate(p.contents, cutoff))
            return XS_OK
        except Exception as e:  # report through the status code
            err.append(e)
            return XS_EINVAL

    fn = EVAL_FN(cb)
    r = xs_tune_result()
    st = load_library().xs_tune_search(built_grids, ctypes.byref(cfg), fn,
                                       None, ctypes.byref(r))
    if err:
        raise err[0]
    _check(st, "xs_tune_search")
    return r


def xs_tune(tables: Tables, E, mat, cfg: xs_tune_config = None, out=None,
            workspace=None, stream=None, sizes=None, cache_path=None,
            active=None):
    """Tune xs_lookup_batch (or, with an active mask, xs_lookup_active) on
    these sample queries and record the winners in the handle.  sizes: batch
    sizes to tune (each tunes on the first n queries); None tunes len(E) and
    returns its one xs_tune_result, else a list in the order of sizes.
    cache_path: tuned-parameter file read before and written after."""
    import numpy as np
    import torch
    _check_queries(E, mat)
    if cfg is None:
        cfg = xs_tune_config_default()
    single = sizes is None
    sz = np.ascontiguousarray([E.numel()] if single else list(sizes),
                              dtype=np.int64)
    n_max = int(sz.max())
    if n_max > E.numel():
        raise ValueError("a size exceeds the sample queries")
    if active is not None:
        if active.dtype != torch.uint8 or active.numel() < n_max:
            raise TypeError("active must be a uint8 tensor covering the sizes")
        cfg.active = 1
    dt = torch.float64 if cfg.precision == XS_FP64 else torch.float32
    if out is None:
        out = torch.empty((n_max, XS_CHANNELS), dtype=dt, device=E.device)
    if workspace is None:
        nb = xs_workspace_size(tables, n_max, make_params(
            cfg.precision, grid=XS_GRID_NUCLIDE, sort=XS_SORT_BAND_MATERIAL,
            sort_threshold=0))
        keep, ws, nb = _workspace(nb, E.device)
    else:
        keep, ws, nb = workspace
    req = xs_tune_request(
        len(sz), 0, sz.ctypes.data, E.data_ptr(), mat.data_ptr(),
        active.data_ptr() if active is not None else None, out.data_ptr(),
        ws.value if ws is not None else None, nb,
        _stream_ptr(stream, E.device).value,
        cache_path.encode() if cache_path else None, cfg)
    res = (xs_tune_result * len(sz))()
    _check(load_library().xs_tune(tables.handle, ctypes.byref(req), res),
           "xs_tune")
    return res[0] if single else list(res)


def xs_set_tuned(tables: Tables, n: int, params: xs_params = None,
                 active: bool = False):
    _check(load_library().xs_set_tuned(
        tables.handle, n, 1 if active else 0,
        ctypes.byref(params) if params is not None else None),
        "xs_set_tuned")


def xs_tune_load(tables: Tables, cache_path: str) -> int:
    """Load the entries of a tuned-parameter file that match this handle and
    device; returns how many."""
    n = ctypes.c_int32()
    _check(load_library().xs_tune_load(tables.handle, cache_path.encode(),
                                       ctypes.byref(n)), "xs_tune_load")
    return n.value


def xs_tune_key_of(tables: Tables, precision: int, active: bool, n: int) -> xs_tune_key:
    k = xs_tune_key()
    _check(load_library().xs_tune_key_of(tables.handle, precision,
                                         1 if active else 0, n,
                                         ctypes.byref(k)), "xs_tune_key_of")
    return k


def make_tune_key(device: str, checksum: int, precision: int, active: bool,
                  n: int) -> xs_tune_key:
    """A key built on the host (no device), for xs_tune_cache_get/put."""
    k = xs_tune_key()
    k.device = device.encode()
    k.checksum = checksum
    k.precision = precision
    k.active = 1 if active else 0
    k.size_class = max(int(n), 1).bit_length() - 1
    return k


def xs_tune_cache_get(cache_path: str, key: xs_tune_key):
    """(params, best_ms) of the key's entry, or None if the file has none."""
    p = xs_params()
    ms = ctypes.c_double()
    st = load_library().xs_tune_cache_get(cache_path.encode(), ctypes.byref(key),
                                          ctypes.byref(p), ctypes.byref(ms))
    if st == XS_ENOTBUILT:
        return None
    _check(st, "xs_tune_cache_get")
    return p, ms.value


def xs_tune_cache_put(cache_path: str, key: xs_tune_key, params: xs_params,
                      best_ms: float):
    _check(load_library().xs_tune_cache_put(cache_path.encode(),
                                            ctypes.byref(key),
                                            ctypes.byref(params), best_ms),
           "xs_tune_cache_put")


class Stream:
    """Owns an xs_stream_t (persistent-kernel request stream)."""

    def __init__(self, handle: ctypes.c_void_p, max_requests: int):
        self.handle = handle
        self.max_requests = max_requests
        self._keep = None
        self._count = 0

    def close(self):
        if self.handle and self.handle.value:
            _check(load_library().xs_stream_destroy(self.handle),
                   "xs_stream_destroy")
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def xs_stream_create(tables: Tables, params: xs_params = None,
                     max_requests: int = 4096, stream=None) -> Stream:
    import torch
    h = ctypes.c_void_p()
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(load_library().xs_stream_create(
        tables.handle, ctypes.byref(params) if params is not None else None,
        max_requests, ctypes.c_void_p(s.cuda_stream), ctypes.byref(h)),
        "xs_stream_create")
    return Stream(h, max_requests)


def xs_stream_submit(stream: Stream, requests):
    """requests: list of (E, mat, out) device tensors (out [n, 5] of the
    stream's precision)."""
    arr = (xs_request * len(requests))()
    for i, (E, mat, out) in enumerate(requests):
        _check_queries(E, mat)
        if out.shape[0] < E.numel() or not out.is_contiguous():
            raise ValueError("out must be a contiguous [n, 5] tensor")
        arr[i] = xs_request(E.numel(), E.data_ptr(), mat.data_ptr(),
                            out.data_ptr())
    stream._keep = list(requests)
    stream._count = len(requests)
    _check(load_library().xs_stream_submit(stream.handle, arr, len(requests)),
           "xs_stream_submit")


def xs_stream_wait(stream: Stream):
    """Returns (stats list of dicts, makespan_us)."""
    stats = (xs_request_stats * max(stream._count, 1))()
    mk = ctypes.c_double()
    _check(load_library().xs_stream_wait(stream.handle, stats, ctypes.byref(mk)),
           "xs_stream_wait")
    out = [dict(n=s.n, start_us=s.start_us, end_us=s.end_us,
                latency_us=s.latency_us) for s in stats[:stream._count]]
    stream._keep = None
    return out, mk.value


def xs_stream_params(stream: Stream) -> xs_params:
    p = xs_params()
    _check(load_library().xs_stream_params(stream.handle, ctypes.byref(p)),
           "xs_stream_params")
    return p


def xs_stream_destroy(stream: Stream):
    stream.close()


class RequestBatch:
    """Workspace and descriptors of one xs_lookup_requests call."""

    def __init__(self, nbytes: int, device):
        self.keep, self.ptr, self.nbytes = _workspace(nbytes, device)
        self.requests = None
        self.n_req = 0


def _request_array(requests):
    arr = (xs_request * len(requests))()
    for i, (E, mat, out) in enumerate(requests):
        _check_queries(E, mat)
        if out.shape[0] < E.numel() or not out.is_contiguous():
            raise ValueError("out must be a contiguous [n, 5] tensor")
        arr[i] = xs_request(E.numel(), E.data_ptr(), mat.data_ptr(),
                            out.data_ptr())
    return arr


def xs_requests_workspace_size(tables: Tables, requests,
                               params: xs_params = None) -> int:
    arr = _request_array(requests)
    b = ctypes.c_size_t()
    _check(load_library().xs_requests_workspace_size(
        tables.handle, arr, len(requests),
        ctypes.byref(params) if params is not None else None, ctypes.byref(b)),
        "xs_requests_workspace_size")
    return b.value


def xs_lookup_requests(tables: Tables, requests, params: xs_params = None,
                       batch: RequestBatch = None, stream=None) -> RequestBatch:
    """requests: list of (E, mat, out) device tensors.  Returns the batch
    object holding the workspace (pass it to xs_requests_stats, or back in
    to reuse its workspace)."""
    if not requests:
        raise ValueError("no requests")
    dev = requests[0][0].device
    arr = _request_array(requests)
    lib = load_library()
    pp = ctypes.byref(params) if params is not None else None
    need = ctypes.c_size_t()
    _check(lib.xs_requests_workspace_size(tables.handle, arr, len(requests), pp,
                                          ctypes.byref(need)),
           "xs_requests_workspace_size")
    if batch is None or batch.nbytes < need.value:
        batch = RequestBatch(need.value, dev)
    batch.requests = list(requests)
    batch.n_req = len(requests)
    _check(lib.xs_lookup_requests(tables.handle, arr, len(requests), pp,
                                  batch.ptr, batch.nbytes,
                                  _stream_ptr(stream, dev)),
           "xs_lookup_requests")
    return batch


def xs_requests_stats(batch: RequestBatch, stream=None):
    """Synchronises and returns (stats list of dicts, makespan_us)."""
    n = batch.n_req
    stats = (xs_request_stats * n)()
    mk = ctypes.c_double()
    dev = batch.requests[0][0].device
    _check(load_library().xs_requests_stats(batch.ptr, n,
                                            _stream_ptr(stream, dev), stats,
                                            ctypes.byref(mk)),
           "xs_requests_stats")
    return [dict(n=s.n, start_us=s.start_us, end_us=s.end_us,
                 latency_us=s.latency_us) for s in stats], mk.value


def xs_event_run(tables: Tables, n_slots: int, n_histories: int, seed: int,
                 params: xs_params = None, e_cut: float = 1e-5,
                 check_every: int = 8, max_iterations: int = 1 << 20,
                 device="cuda:0", stream=None, workspace=None):
    """Runs the toy event loop; returns (result dict, tallies dict of
    device tensors: collisions int32, energy float64, fate uint8, each
    [n_histories])."""
    import torch
    prec = XS_FP64 if params is None else params.precision
    if prec == XS_AUTO:
        prec = XS_FP64
    dt = torch.float64 if prec == XS_FP64 else torch.float32
    dev = torch.device(device)
    buf = {
        "E": torch.empty(n_slots, dtype=torch.float64, device=dev),
        "mat": torch.empty(n_slots, dtype=torch.int32, device=dev),
        "alive": torch.zeros(n_slots, dtype=torch.uint8, device=dev),
        "hist": torch.empty(n_slots, dtype=torch.int64, device=dev),
        "ncoll": torch.empty(n_slots, dtype=torch.int32, device=dev),
        "sigma": torch.empty((n_slots, XS_CHANNELS), dtype=dt, device=dev),
        "counters": torch.zeros(3, dtype=torch.int64, device=dev),
        "t_collisions": torch.zeros(max(n_histories, 1), dtype=torch.int32,
                                    device=dev),
        "t_energy": torch.zeros(max(n_histories, 1), dtype=torch.float64,
                                device=dev),
        "t_fate": torch.zeros(max(n_histories, 1), dtype=torch.uint8,
                              device=dev),
    }
    b = xs_event_buffers(*[buf[f].data_ptr() for f, _ in
                           xs_event_buffers._fields_])
    cfg = xs_event_config(n_slots, n_histories, seed, e_cut, check_every,
                          max_iterations)
    pp = ctypes.byref(params) if params is not None else None
    lib = load_library()
    if workspace is None:
        nb = ctypes.c_size_t()
        _check(lib.xs_event_workspace_size(tables.handle, ctypes.byref(cfg), pp,
                                           ctypes.byref(nb)),
               "xs_event_workspace_size")
        keep, ws, nb = _workspace(nb.value, dev)
    else:
        keep, ws, nb = workspace
    r = xs_event_result()
    _check(lib.xs_event_run(tables.handle, ctypes.byref(cfg), ctypes.byref(b),
                            pp, ws, nb, _stream_ptr(stream, dev),
                            ctypes.byref(r)), "xs_event_run")
    res = {f: getattr(r, f) for f, _ in xs_event_result._fields_}
    tallies = {"collisions": buf["t_collisions"][:n_histories],
               "energy": buf["t_energy"][:n_histories],
               "fate": buf["t_fate"][:n_histories]}
    return res, tallies
