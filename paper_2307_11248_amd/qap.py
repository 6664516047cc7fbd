"""Python binding of libqap (the C ABI in include/qap.h): argument marshalling only.

Every computation runs in the HIP library.  If ``libqap.so`` has not been built the
first call raises ``RuntimeError``; there is no CPU fallback.

Host functions take and return numpy arrays.  The ``*_async`` functions take torch
tensors that live on the GPU and enqueue work on a torch stream (the current one by
default); torch is used for device memory and streams only.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libqap.so")

QAP_OK = 0
QAP_E_INVALID = -1
QAP_E_NOT_PERM = -2
QAP_E_RANGE = -3
QAP_E_DEVICE = -4
QAP_E_NOMEM = -5
QAP_E_BUSY = -6
QAP_E_UNSUPPORTED = -7
QAP_E_SCRATCH = -8
QAP_NOALLOC_SCRATCH_BYTES = 64 << 20
QAP_NMAX = 512
QAP_NMAX_BATCH = 512   # batched and served searches

EXPORTS = [
    "qap_strerror", "qap_create", "qap_destroy", "qap_size", "qap_cost", "qap_cost_async", "qap_delta_table",
    "qap_delta_table_async", "qap_2opt", "qap_2opt_async", "qap_tabu", "qap_tabu_async", "qap_tabu_noalloc_async",
    "qap_tabu_freq_async", "qap_tabu_trace_async",
    "qap_tabu_plain_async", "qap_2opt_with_table_async", "qap_tabu_with_table_async", "qap_set_tile_rows",
    "qap_get_tile_rows", "qap_launch_tile_rows", "qap_batch_create", "qap_batch_create_freq", "qap_batch_freq_async", "qap_batch_size", "qap_batch_groups",
    "qap_batch_run_async",
    "qap_batch_tables_async", "qap_batch_search_async", "qap_batch_destroy", "qap_tabu_batch",
    "qap_tabu_batch_concat",
    "qap_tune_tile_rows", "qap_server_create", "qap_server_footprint", "qap_server_submit",
    "qap_server_submit_matrices", "qap_server_submit_freq", "qap_server_poll_freq", "qap_server_set_queue_limit", "qap_server_step", "qap_server_start",
    "qap_server_stop", "qap_server_poll", "qap_server_result", "qap_server_cancel", "qap_server_inject_failure",
    "qap_server_stats", "qap_server_destroy",
]

ALGOS = {"tabu": 0, "2opt": 1, "batch": 2}

_lib = None
_lock = threading.Lock()
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_vp = ctypes.c_void_p


class QapError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, lib().qap_strerror(code).decode(), code))


def lib():
    """Load libqap.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libqap.so is not built: run `python -m paper_2307_11248_amd.build` "
                                   "(or __graft_entry__.build()) first")
            L = ctypes.CDLL(LIB_PATH)
            i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
            sig = {
                "qap_strerror": (ctypes.c_char_p, [ctypes.c_int]),
                "qap_create": (ctypes.c_int, [_i32p, _i32p, i32, ctypes.POINTER(_vp)]),
                "qap_destroy": (ctypes.c_int, [_vp]),
                "qap_size": (ctypes.c_int, [_vp]),
                "qap_cost": (ctypes.c_int, [_vp, _i32p, i32, _i64p]),
                "qap_cost_async": (ctypes.c_int, [_vp, _vp, i32, _vp, _vp]),
                "qap_delta_table": (ctypes.c_int, [_vp, _i32p, i32, _i32p]),
                "qap_delta_table_async": (ctypes.c_int, [_vp, _vp, i32, _vp, _vp]),
                "qap_2opt": (ctypes.c_int, [_vp, _i32p, i32, i32, _i64p, _i32p]),
                "qap_2opt_async": (ctypes.c_int, [_vp, _vp, i32, i32, _vp, _vp, _vp]),
                "qap_tabu": (ctypes.c_int, [_vp, _i32p, i32, i32, i32, i32, u64, _i64p, _i32p]),
                "qap_tabu_async": (ctypes.c_int, [_vp, _vp, i32, i32, i32, i32, u64, i64, _vp, _vp, _vp]),
                "qap_tabu_noalloc_async": (ctypes.c_int, [_vp, _vp, i32, i32, i32, i32, u64, i64, _vp, _vp,
                                                          _vp]),
                "qap_tabu_freq_async": (ctypes.c_int, [_vp, _vp, i32, i32, i32, i32, u64, i64, i32, i32, _vp,
                                                        _vp, _vp, _vp]),
                "qap_tabu_trace_async": (ctypes.c_int, [_vp, _vp, i32, i32, i32, i32, u64, i64, i32, i32, _vp,
                                                        _vp, _vp, _vp, i32, _vp]),
                "qap_tabu_plain_async": (ctypes.c_int, [_vp, _vp, i32, i32, i32, i32, u64, i64, _vp, _vp,
                                                        _vp]),
                "qap_2opt_with_table_async": (ctypes.c_int, [_vp, _vp, _vp, i32, i32, _vp, _vp, _vp]),
                "qap_tabu_with_table_async": (ctypes.c_int, [_vp, _vp, _vp, i32, i32, i32, i32, u64, i64, _vp,
                                                             _vp, _vp]),
                "qap_set_tile_rows": (ctypes.c_int, [_vp, i32, i32]),
                "qap_get_tile_rows": (ctypes.c_int, [_vp, i32, _i32p]),
                "qap_launch_tile_rows": (ctypes.c_int, [_vp, i32, i32, _i32p]),
                "qap_tune_tile_rows": (ctypes.c_int, [_vp, i32, i32, i32, ctypes.POINTER(ctypes.c_float)]),
                "qap_server_create": (ctypes.c_int, [i64, i32, ctypes.c_double, ctypes.POINTER(_vp)]),
                "qap_server_footprint": (i64, [_vp, i32, i32]),
                "qap_server_submit": (ctypes.c_int, [_vp, _vp, _i32p, i32, i32, i32, u64, _i64p]),
                "qap_server_submit_matrices": (ctypes.c_int, [_vp, _i32p, _i32p, i32, _i32p, i32, i32, i32, u64,
                                                              _i64p]),
                "qap_server_submit_freq": (ctypes.c_int, [_vp, _vp, _i32p, i32, i32, i32, u64, i32, i32, _i64p]),
                "qap_server_poll_freq": (ctypes.c_int, [_vp, i64, _i32p, _i64p, _i32p]),
                "qap_server_set_queue_limit": (ctypes.c_int, [_vp, i32]),
                "qap_server_step": (ctypes.c_int, [_vp, _i32p, _i32p]),
                "qap_server_start": (ctypes.c_int, [_vp]),
                "qap_server_stop": (ctypes.c_int, [_vp]),
                "qap_server_poll": (ctypes.c_int, [_vp, i64, _i32p, _i64p]),
                "qap_server_cancel": (ctypes.c_int, [_vp, i64]),
                "qap_server_inject_failure": (ctypes.c_int, [_vp, i64]),
                "qap_server_result": (ctypes.c_int, [_vp, i64, _i32p, _i64p, _i32p,
                                                     ctypes.POINTER(ctypes.c_double)]),
                "qap_server_stats": (ctypes.c_int, [_vp, _i64p]),
                "qap_server_destroy": (ctypes.c_int, [_vp]),
                "qap_batch_create": (ctypes.c_int, [ctypes.POINTER(_vp), i32, _i32p, i32, _i32p, _i32p, _u64p,
                                                    _i32p, ctypes.POINTER(_vp)]),
                "qap_batch_create_freq": (ctypes.c_int, [ctypes.POINTER(_vp), i32, _i32p, i32, _i32p, _i32p, _u64p,
                                                         _i32p, _i32p, _i32p, ctypes.POINTER(_vp)]),
                "qap_batch_freq_async": (ctypes.c_int, [_vp, _vp, _vp]),
                "qap_batch_size": (ctypes.c_int, [_vp, _i64p, _i64p]),
                "qap_batch_groups": (ctypes.c_int, [_vp, _i32p]),
                "qap_batch_run_async": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
                "qap_batch_tables_async": (ctypes.c_int, [_vp, _vp, _vp]),
                "qap_batch_search_async": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
                "qap_batch_destroy": (ctypes.c_int, [_vp]),
                "qap_tabu_batch": (ctypes.c_int, [ctypes.POINTER(_vp), i32, ctypes.POINTER(_i32p), _i32p, i32,
                                                  _i32p, _i32p, _u64p, ctypes.POINTER(_i64p)]),
                "qap_tabu_batch_concat": (ctypes.c_int, [ctypes.POINTER(_vp), i32, _i32p, _i32p, i32, _i32p,
                                                         _i32p, _u64p, _i64p, _i32p]),
            }
            for name, (res, args) in sig.items():
                f = getattr(L, name)
                f.restype, f.argtypes = res, args
            _lib = L
    return _lib


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise QapError(rc, what)
    return rc


def _check_rows(rc: int, what: str) -> int:
    """Tile rows are returned as 1, 2, 4, 8, 16 or -8 (the streamed kernel); other negative
    values are error codes."""
    if rc < 0 and rc != -8:
        raise QapError(rc, what)
    return rc


def _arr(a, dtype, shape=None):
    a = np.ascontiguousarray(a, dtype=dtype)
    if shape is not None and a.shape != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (tuple(shape), a.shape))
    return a


def _ptr(a, t):
    return a.ctypes.data_as(t)


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))


def _dptr(t, dtype_name):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous() or str(t.dtype) != "torch." + dtype_name:
        raise ValueError("expected a contiguous %s tensor on the GPU" % dtype_name)
    return ctypes.c_void_p(t.data_ptr())


class Handle:
    """One QAP instance (F, D) copied to the current HIP device (``qap_create``)."""

    def __init__(self, F, D):
        F = _arr(F, np.int32)
        n = F.shape[0]
        D = _arr(D, np.int32, (n, n))
        if F.shape != (n, n):
            raise ValueError("F must be square")
        h = _vp()
        _check(lib().qap_create(_ptr(F, _i32p), _ptr(D, _i32p), n, ctypes.byref(h)), "qap_create")
        self._h = h
        self.n = n
        self.m = n * (n - 1) // 2
        self.sym = bool((F == F.T).all() and (D == D.T).all())

    @property
    def ptr(self):
        if self._h is None:
            raise ValueError("handle is closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().qap_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- tile shape (thread configuration); algo is "tabu", "2opt" or "batch"
    def set_tile_rows(self, algo: str, rows: int):
        _check(lib().qap_set_tile_rows(self.ptr, ALGOS[algo], int(rows)), "qap_set_tile_rows")

    def tile_rows(self, algo: str):
        lanes = ctypes.c_int32(0)
        rows = _check_rows(lib().qap_get_tile_rows(self.ptr, ALGOS[algo], ctypes.byref(lanes)), "qap_get_tile_rows")
        return rows, lanes.value

    def launch_tile_rows(self, algo: str, k: int):
        """(rows, lanes per search) that a launch of k starts uses (``qap_launch_tile_rows``)."""
        lanes = ctypes.c_int32(0)
        rows = _check_rows(lib().qap_launch_tile_rows(self.ptr, ALGOS[algo], int(k), ctypes.byref(lanes)),
                           "qap_launch_tile_rows")
        return rows, lanes.value

    def tune_tile_rows(self, algo: str, k: int = 256, iters: int = 300):
        """Time every fitting shape on the device and keep the fastest (``qap_tune_tile_rows``).
        Returns (rows, {rows: ms} for the shapes that fit)."""
        ms = (ctypes.c_float * 6)()
        rows = _check_rows(lib().qap_tune_tile_rows(self.ptr, ALGOS[algo], int(k), int(iters), ms),
                           "qap_tune_tile_rows")
        return rows, {r: float(t) for r, t in zip((1, 2, 4, 8, 16, -8), ms) if t >= 0}

    # -- blocking host calls
    def cost(self, perms) -> np.ndarray:
        perms = _arr(perms, np.int32)
        perms = perms.reshape(-1, self.n)
        k = perms.shape[0]
        out = np.zeros(k, dtype=np.int64)
        _check(lib().qap_cost(self.ptr, _ptr(perms, _i32p), k, _ptr(out, _i64p)), "qap_cost")
        return out

    def delta_table(self, perms) -> np.ndarray:
        perms = _arr(perms, np.int32).reshape(-1, self.n)
        k = perms.shape[0]
        out = np.zeros((k, self.m), dtype=np.int32)
        _check(lib().qap_delta_table(self.ptr, _ptr(perms, _i32p), k, _ptr(out, _i32p)), "qap_delta_table")
        return out

    def two_opt(self, perms, max_iters: int = 0):
        p = np.array(perms, dtype=np.int32, copy=True).reshape(-1, self.n)
        k = p.shape[0]
        costs = np.zeros(k, dtype=np.int64)
        steps = np.zeros(k, dtype=np.int32)
        _check(lib().qap_2opt(self.ptr, _ptr(p, _i32p), k, int(max_iters), _ptr(costs, _i64p),
                              _ptr(steps, _i32p)), "qap_2opt")
        return p, costs, steps

    def tabu(self, perms, iters: int, lo: int, hi: int, seed: int):
        p = np.array(perms, dtype=np.int32, copy=True).reshape(-1, self.n)
        k = p.shape[0]
        costs = np.zeros(k, dtype=np.int64)
        done = np.zeros(k, dtype=np.int32)
        _check(lib().qap_tabu(self.ptr, _ptr(p, _i32p), k, int(iters), int(lo), int(hi), int(seed),
                              _ptr(costs, _i64p), _ptr(done, _i32p)), "qap_tabu")
        return p, costs, done

    # -- device / stream calls (torch tensors)
    def cost_async(self, d_perms, d_costs, stream=None):
        _check(lib().qap_cost_async(self.ptr, _dptr(d_perms, "int32"), d_perms.shape[0],
                                    _dptr(d_costs, "int64"), _stream_ptr(stream)), "qap_cost_async")

    def delta_table_async(self, d_perms, d_table, stream=None):
        _check(lib().qap_delta_table_async(self.ptr, _dptr(d_perms, "int32"), d_perms.shape[0],
                                           _dptr(d_table, "int32"), _stream_ptr(stream)),
               "qap_delta_table_async")

    def two_opt_async(self, d_perms, d_costs, d_steps=None, max_iters: int = 0, stream=None):
        _check(lib().qap_2opt_async(self.ptr, _dptr(d_perms, "int32"), d_perms.shape[0], int(max_iters),
                                    _dptr(d_costs, "int64"), _dptr(d_steps, "int32"), _stream_ptr(stream)),
               "qap_2opt_async")

    def tabu_async(self, d_perms, iters, lo, hi, seed, d_best, d_done=None, start_base: int = 0,
                   stream=None, plain: bool = False):
        f = lib().qap_tabu_plain_async if plain else lib().qap_tabu_async
        _check(f(self.ptr, _dptr(d_perms, "int32"), d_perms.shape[0], int(iters), int(lo), int(hi), int(seed),
                 int(start_base), _dptr(d_best, "int64"), _dptr(d_done, "int32"), _stream_ptr(stream)),
               "qap_tabu_async")

    def tabu_noalloc_async(self, d_perms, iters, lo, hi, seed, d_best, d_done=None, start_base: int = 0,
                           stream=None):
        """tabu_async with its scratch taken from the library's fixed device array
        (``qap_tabu_noalloc_async``); raises QapError(QAP_E_SCRATCH) if it would not fit."""
        _check(lib().qap_tabu_noalloc_async(self.ptr, _dptr(d_perms, "int32"), d_perms.shape[0], int(iters),
                                            int(lo), int(hi), int(seed), int(start_base), _dptr(d_best, "int64"),
                                            _dptr(d_done, "int32"), _stream_ptr(stream)),
               "qap_tabu_noalloc_async")

    def tabu_freq_async(self, d_perms, iters, lo, hi, seed, d_best, d_freq, d_done=None, start_base: int = 0,
                        div: int = 0, attr: int = 0, stream=None):
        """tabu_async that also fills d_freq (int32[k][n(n-1)/2]) with the number of
        exchanges of each pair of locations, and with div > 0 makes the frequency-based
        diversification move; attr 1 makes the units moved tabu instead of the pair of
        locations, attr 2 the return of both units to locations they left
        (``qap_tabu_freq_async``)."""
        _check(lib().qap_tabu_freq_async(self.ptr, _dptr(d_perms, "int32"), d_perms.shape[0], int(iters), int(lo),
                                         int(hi), int(seed), int(start_base), int(div), int(attr),
                                         _dptr(d_best, "int64"),
                                         _dptr(d_done, "int32"), _dptr(d_freq, "int32"), _stream_ptr(stream)),
               "qap_tabu_freq_async")

    def tabu_trace_async(self, d_perms, iters, lo, hi, seed, d_best, d_freq, d_trace, d_done=None,
                         start_base: int = 0, div: int = 0, attr: int = 0, stream=None):
        """tabu_freq_async that also records the first d_trace.shape[1] moves of every start
        as (r, s, delta, cost after) into d_trace (int64[k][cap][4]) (``qap_tabu_trace_async``)."""
        cap = int(d_trace.shape[1]) if d_trace.dim() == 3 else 0
        if d_trace.dim() != 3 or d_trace.shape[0] != d_perms.shape[0] or d_trace.shape[2] != 4:
            raise ValueError("d_trace must be int64[k][cap][4]")
        _check(lib().qap_tabu_trace_async(self.ptr, _dptr(d_perms, "int32"), d_perms.shape[0], int(iters), int(lo),
                                          int(hi), int(seed), int(start_base), int(div), int(attr),
                                          _dptr(d_best, "int64"), _dptr(d_done, "int32"), _dptr(d_freq, "int32"),
                                          _dptr(d_trace, "int64"), cap, _stream_ptr(stream)),
               "qap_tabu_trace_async")

    def two_opt_with_table_async(self, d_perms, d_table, d_costs, d_steps=None, max_iters: int = 0, stream=None):
        _check(lib().qap_2opt_with_table_async(self.ptr, _dptr(d_perms, "int32"), _dptr(d_table, "int32"),
                                               d_perms.shape[0], int(max_iters), _dptr(d_costs, "int64"),
                                               _dptr(d_steps, "int32"), _stream_ptr(stream)),
               "qap_2opt_with_table_async")

    def tabu_with_table_async(self, d_perms, d_table, iters, lo, hi, seed, d_best, d_done=None,
                              start_base: int = 0, stream=None):
        _check(lib().qap_tabu_with_table_async(self.ptr, _dptr(d_perms, "int32"), _dptr(d_table, "int32"),
                                               d_perms.shape[0], int(iters), int(lo), int(hi), int(seed),
                                               int(start_base), _dptr(d_best, "int64"), _dptr(d_done, "int32"),
                                               _stream_ptr(stream)),
               "qap_tabu_with_table_async")


def _batch_args(handles, ks, lo, hi, seeds):
    m = len(handles)
    hs = (_vp * max(m, 1))(*[h.ptr for h in handles])
    ks = _arr(ks, np.int32, (m,))
    lo = _arr(lo, np.int32, (m,))
    hi = _arr(hi, np.int32, (m,))
    seeds = _arr(seeds, np.uint64, (m,))
    return m, hs, ks, lo, hi, seeds


class Batch:
    """A planned batch of tabu searches over many instances (``qap_batch_create``).

    Instance i (``handles[i]``) runs ``ks[i]`` starts with tenure range [lo[i], hi[i]]
    and seed seeds[i]; starts and results are concatenated in instance order.

    With ``freq=True`` every search keeps the frequency memory and may use the extensions
    of ``tabu_freq_async`` (``div`` and ``attr`` per instance, or None for 0):
    ``qap_batch_create_freq``; ``freq_async`` copies the counts out.
    """

    def __init__(self, handles, ks, iters, lo, hi, seeds, rows=None, freq=False, div=None, attr=None):
        m, hs, ks, lo, hi, seeds = _batch_args(handles, ks, lo, hi, seeds)
        rows_p = None if rows is None else _ptr(_arr(rows, np.int32, (m,)), _i32p)
        b = _vp()
        self.freq_ints = 0
        if freq:
            div_a = None if div is None else _arr(div, np.int32, (m,))
            attr_a = None if attr is None else _arr(attr, np.int32, (m,))
            _check(lib().qap_batch_create_freq(hs, m, _ptr(ks, _i32p), int(iters), _ptr(lo, _i32p), _ptr(hi, _i32p),
                                               _ptr(seeds, _u64p), rows_p,
                                               None if div_a is None else _ptr(div_a, _i32p),
                                               None if attr_a is None else _ptr(attr_a, _i32p), ctypes.byref(b)),
                   "qap_batch_create_freq")
            self.freq_ints = int(sum(int(k) * h.m for k, h in zip(ks, handles)))
        else:
            if div is not None or attr is not None:
                raise ValueError("div and attr need freq=True")
            _check(lib().qap_batch_create(hs, m, _ptr(ks, _i32p), int(iters), _ptr(lo, _i32p), _ptr(hi, _i32p),
                                          _ptr(seeds, _u64p), rows_p, ctypes.byref(b)), "qap_batch_create")
        self._b = b
        self._handles = list(handles)   # the plan refers to their device matrices
        s, p = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib().qap_batch_size(b, ctypes.byref(s), ctypes.byref(p)), "qap_batch_size")
        self.starts, self.perm_ints = s.value, p.value

    def run_async(self, d_perms, d_best, d_done=None, stream=None):
        _check(lib().qap_batch_run_async(self._b, _dptr(d_perms, "int32"), _dptr(d_best, "int64"),
                                         _dptr(d_done, "int32"), _stream_ptr(stream)), "qap_batch_run_async")

    def groups(self, counts: bool = False):
        """Kernel dispatches of one search phase (one per tile-shape variant in use); with
        counts=True also the searches per variant (int32[9], the header's order)."""
        c = np.zeros(9, dtype=np.int32)
        g = _check(lib().qap_batch_groups(self._b, _ptr(c, _i32p)), "qap_batch_groups")
        return (g, c) if counts else g

    def freq_async(self, d_freq, stream=None):
        """Copy the frequency memory of the last run (int32[sum k_i m_i], instance order,
        start order, packed pair order) into d_freq (``qap_batch_freq_async``)."""
        _check(lib().qap_batch_freq_async(self._b, _dptr(d_freq, "int32"), _stream_ptr(stream)),
               "qap_batch_freq_async")

    def tables_async(self, d_perms, stream=None):
        _check(lib().qap_batch_tables_async(self._b, _dptr(d_perms, "int32"), _stream_ptr(stream)),
               "qap_batch_tables_async")

    def search_async(self, d_perms, d_best, d_done=None, stream=None):
        _check(lib().qap_batch_search_async(self._b, _dptr(d_perms, "int32"), _dptr(d_best, "int64"),
                                            _dptr(d_done, "int32"), _stream_ptr(stream)), "qap_batch_search_async")

    def close(self):
        if getattr(self, "_b", None) is not None:
            lib().qap_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def tabu_batch(handles, perms, ks, iters, lo, hi, seeds):
    """Blocking batched tabu (``qap_tabu_batch_concat``): perms is the concatenation of every
    instance's starts, flattened; returns (best permutations, best costs, moves made)."""
    m, hs, ks, lo, hi, seeds = _batch_args(handles, ks, lo, hi, seeds)
    p = np.array(perms, dtype=np.int32, copy=True).reshape(-1)
    total = int(sum(int(k) for k in ks))
    best = np.zeros(total, dtype=np.int64)
    done = np.zeros(total, dtype=np.int32)
    _check(lib().qap_tabu_batch_concat(hs, m, _ptr(p, _i32p), _ptr(ks, _i32p), int(iters), _ptr(lo, _i32p),
                                       _ptr(hi, _i32p), _ptr(seeds, _u64p), _ptr(best, _i64p), _ptr(done, _i32p)),
           "qap_tabu_batch_concat")
    return p, best, done


def tabu_batch_lists(handles, perms_list, iters, lo, hi, seeds):
    """Blocking batched tabu with per-instance arrays (``qap_tabu_batch``): perms_list[i] is
    instance i's starts, int32[k_i][n_i]; returns (list of best permutations, list of best
    costs)."""
    ks = [len(p) for p in perms_list]
    m, hs, ks_a, lo, hi, seeds = _batch_args(handles, ks, lo, hi, seeds)
    ps = [np.array(p, dtype=np.int32, copy=True).reshape(k, h.n) for p, k, h in zip(perms_list, ks, handles)]
    bs = [np.zeros(k, dtype=np.int64) for k in ks]
    pp = (_i32p * max(m, 1))(*[_ptr(p, _i32p) for p in ps])
    bp = (_i64p * max(m, 1))(*[_ptr(b, _i64p) for b in bs])
    _check(lib().qap_tabu_batch(hs, m, pp, _ptr(ks_a, _i32p), int(iters), _ptr(lo, _i32p), _ptr(hi, _i32p),
                                _ptr(seeds, _u64p), bp), "qap_tabu_batch")
    return ps, bs


class Server:
    """Continuous-batching tabu server (``qap_server_*``): submit requests, drive it with
    step() (or start() its own thread), collect results by ticket with poll() or result()."""

    def __init__(self, pool_bytes: int = 1 << 30, max_active: int = 256, chunk_ms: float = 2.0):
        s = _vp()
        _check(lib().qap_server_create(int(pool_bytes), int(max_active), float(chunk_ms), ctypes.byref(s)),
               "qap_server_create")
        self._s = s
        self._n = {}

    def footprint(self, n: int, sym: bool = False) -> int:
        """Device bytes a request of size n with its own matrices takes from the pool while admitted."""
        return _check(lib().qap_server_footprint(self._s, int(n), int(bool(sym))), "qap_server_footprint")

    def submit(self, F, D, start, iters: int, lo: int, hi: int, seed: int) -> int:
        """A request with its own F and D (qap_server_submit_matrices); returns its ticket."""
        F = _arr(F, np.int32)
        n = F.shape[0]
        D = _arr(D, np.int32, (n, n))
        start = _arr(start, np.int32, (n,))
        t = ctypes.c_int64(0)
        _check(lib().qap_server_submit_matrices(self._s, _ptr(F, _i32p), _ptr(D, _i32p), n, _ptr(start, _i32p),
                                                int(iters), int(lo), int(hi), int(seed), ctypes.byref(t)),
               "qap_server_submit_matrices")
        self._n[t.value] = n
        return t.value

    def submit_handle(self, h: "Handle", start, iters: int, lo: int, hi: int, seed: int) -> int:
        """A request on an existing handle (qap_server_submit); h must outlive the request."""
        start = _arr(start, np.int32, (h.n,))
        t = ctypes.c_int64(0)
        _check(lib().qap_server_submit(self._s, h.ptr, _ptr(start, _i32p), int(iters), int(lo), int(hi), int(seed),
                                       ctypes.byref(t)), "qap_server_submit")
        self._n[t.value] = h.n
        return t.value

    def submit_freq(self, h: "Handle", start, iters: int, lo: int, hi: int, seed: int, div: int = 0,
                    attr: int = 0) -> int:
        """A request on handle h that keeps the frequency memory and may diversify or use a
        unit attribute (qap_server_submit_freq); collect it with poll_freq."""
        start = _arr(start, np.int32, (h.n,))
        t = ctypes.c_int64(0)
        _check(lib().qap_server_submit_freq(self._s, h.ptr, _ptr(start, _i32p), int(iters), int(lo), int(hi),
                                            int(seed), int(div), int(attr), ctypes.byref(t)),
               "qap_server_submit_freq")
        self._n[t.value] = h.n
        return t.value

    def poll_freq(self, ticket: int):
        """None while queued or running, else (best permutation, best cost, exchange counts)."""
        n = self._n[ticket]
        perm = np.zeros(n, dtype=np.int32)
        freq = np.zeros(max(1, n * (n - 1) // 2), dtype=np.int32)
        best = ctypes.c_int64(0)
        rc = lib().qap_server_poll_freq(self._s, int(ticket), _ptr(perm, _i32p), ctypes.byref(best),
                                        _ptr(freq, _i32p))
        if rc == 0:
            return None
        if rc == 1 or rc == QAP_E_DEVICE:   # collected (or failed): the ticket is forgotten
            del self._n[ticket]
        _check(rc, "qap_server_poll_freq")
        return perm, best.value, freq[:n * (n - 1) // 2]

    def set_queue_limit(self, max_queued: int):
        _check(lib().qap_server_set_queue_limit(self._s, int(max_queued)), "qap_server_set_queue_limit")

    def step(self):
        """One admission + chunk; returns (finished, running, queued)."""
        a, p = ctypes.c_int32(0), ctypes.c_int32(0)
        f = _check(lib().qap_server_step(self._s, ctypes.byref(a), ctypes.byref(p)), "qap_server_step")
        return f, a.value, p.value

    def start(self):
        """Run the server's own stepping thread until stop()."""
        _check(lib().qap_server_start(self._s), "qap_server_start")

    def stop(self):
        _check(lib().qap_server_stop(self._s), "qap_server_stop")

    def poll(self, ticket: int):
        """None while queued or running, else (best permutation, best cost)."""
        n = self._n[ticket]
        perm = np.zeros(n, dtype=np.int32)
        best = ctypes.c_int64(0)
        rc = lib().qap_server_poll(self._s, int(ticket), _ptr(perm, _i32p), ctypes.byref(best))
        if rc == 0:
            return None
        del self._n[ticket]
        _check(rc, "qap_server_poll")
        return perm, best.value

    def result(self, ticket: int):
        """None while queued or running, else (best permutation, best cost, moves, latency ms, queued ms)."""
        n = self._n[ticket]
        perm = np.zeros(n, dtype=np.int32)
        best, moves = ctypes.c_int64(0), ctypes.c_int32(0)
        lat = (ctypes.c_double * 2)()
        rc = lib().qap_server_result(self._s, int(ticket), _ptr(perm, _i32p), ctypes.byref(best),
                                     ctypes.byref(moves), lat)
        if rc == 0:
            return None
        del self._n[ticket]
        _check(rc, "qap_server_result")
        return perm, best.value, moves.value, lat[0], lat[1]

    def cancel(self, ticket: int) -> bool:
        """True if the request was dropped, False if it had already finished."""
        rc = _check(lib().qap_server_cancel(self._s, int(ticket)), "qap_server_cancel")
        if rc == 1:
            del self._n[ticket]
        return rc == 1

    def inject_failure(self, ticket: int):
        """Test hook: corrupt a running request's saved state so that its search fails."""
        _check(lib().qap_server_inject_failure(self._s, int(ticket)), "qap_server_inject_failure")

    def stats(self) -> dict:
        out = np.zeros(9, dtype=np.int64)
        _check(lib().qap_server_stats(self._s, _ptr(out, _i64p)), "qap_server_stats")
        return dict(zip(("running", "queued", "pool_used", "pool_bytes", "steps", "chunks", "finished", "failed",
                         "cancelled"), out.tolist()))

    def close(self):
        if getattr(self, "_s", None) is not None:
            lib().qap_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
