"""CPU oracle for the QAP pairwise-exchange heuristics (Novoa & Qasem, arXiv 2307.11248).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``.  The product package never imports it, and it
shares no code with the HIP path.

The arithmetic lives in ``qap_oracle.c`` (plain C, exact int64); this module compiles
it with gcc and exposes each function through ctypes with numpy arguments.

Functions and the passage each follows:
  cost          Eq. (1)
  delta         Eq. (2) plus the diagonal term the printed equation omits
  delta_table   Sec. 4.1, the whole pairwise-exchange neighbourhood
  delta_update  incremental update of the neighbourhood (Taillard 1991, cited in Sec. 4.3)
  philox        Philox4x64-10 (Salmon et al., SC'11), the tenure generator
  tenure        Sec. 4.3, dynamic tabu-list size
  two_opt       Secs. 4.1-4.2
  tabu          Secs. 4.3-4.4
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qap_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = True) -> str:
    """Compile qap_oracle.c into liboracle.so next to it; return the path."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-Werror",
                               "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            # QAP_ORACLE_LIB names another build of qap_oracle.c (the sanitizer-instrumented
            # one of tests/test_oracle_sanitized.py); by default the library is built here.
            path = os.environ.get("QAP_ORACLE_LIB")
            if not path:
                path = build(force=False)
            lib = ctypes.CDLL(path)
            lib.orc_cost.restype = ctypes.c_int64
            lib.orc_cost.argtypes = [ctypes.c_int, _i32p, _i32p, _i32p]
            lib.orc_delta.restype = ctypes.c_int64
            lib.orc_delta.argtypes = [ctypes.c_int, _i32p, _i32p, _i32p, ctypes.c_int, ctypes.c_int]
            lib.orc_delta_table.restype = None
            lib.orc_delta_table.argtypes = [ctypes.c_int, _i32p, _i32p, _i32p, _i64p]
            lib.orc_delta_table_contraction.restype = None
            lib.orc_delta_table_contraction.argtypes = [ctypes.c_int, _i32p, _i32p, _i32p, _i64p]
            lib.orc_delta_update.restype = None
            lib.orc_delta_update.argtypes = [ctypes.c_int, _i32p, _i32p, _i32p, ctypes.c_int,
                                             ctypes.c_int, _i64p]
            lib.orc_philox4x64_10.restype = None
            lib.orc_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
            lib.orc_tenure.restype = ctypes.c_int32
            lib.orc_tenure.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_int32, ctypes.c_int32]
            lib.orc_2opt.restype = ctypes.c_int
            lib.orc_2opt.argtypes = [ctypes.c_int, _i32p, _i32p, _i32p, ctypes.c_int32, ctypes.c_int,
                                     _i64p, _i32p, _i64p, ctypes.c_int32]
            lib.orc_tabu.restype = ctypes.c_int
            lib.orc_tabu.argtypes = [ctypes.c_int, _i32p, _i32p, _i32p, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                     _i32p, _i64p, _i32p, _i64p, ctypes.c_int32]
            lib.orc_tabu_freq.restype = ctypes.c_int
            lib.orc_tabu_freq.argtypes = [ctypes.c_int, _i32p, _i32p, _i32p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32,
                                          ctypes.c_int32, _i32p, _i64p, _i32p, _i32p, _i64p, ctypes.c_int32]
            _lib = lib
    return _lib


def _mat(a, n):
    a = np.ascontiguousarray(a, dtype=np.int32)
    assert a.shape == (n, n)
    return a


def _vec(a, n):
    a = np.ascontiguousarray(a, dtype=np.int32)
    assert a.shape == (n,)
    return a


def _p32(a):
    return a.ctypes.data_as(_i32p)


def _p64(a):
    return a.ctypes.data_as(_i64p)


def cost(F, D, perm) -> int:
    """Eq. (1) for one permutation."""
    n = len(perm)
    F, D, p = _mat(F, n), _mat(D, n), _vec(perm, n)
    return int(_load().orc_cost(n, _p32(F), _p32(D), _p32(p)))


def delta(F, D, perm, r, s) -> int:
    """Eq. (2) with the diagonal term, for exchanging locations r and s."""
    n = len(perm)
    F, D, p = _mat(F, n), _mat(D, n), _vec(perm, n)
    return int(_load().orc_delta(n, _p32(F), _p32(D), _p32(p), int(r), int(s)))


def delta_table(F, D, perm) -> np.ndarray:
    """All n(n-1)/2 deltas in packed upper-triangle order (int64)."""
    n = len(perm)
    F, D, p = _mat(F, n), _mat(D, n), _vec(perm, n)
    out = np.zeros(n * (n - 1) // 2, dtype=np.int64)
    _load().orc_delta_table(n, _p32(F), _p32(D), _p32(p), _p64(out))
    return out


def delta_table_contraction(F, D, perm) -> np.ndarray:
    """The same table from the contraction form T = G.D^T + G^T.D (G = F[p][p]):
    delta(i, j) = T_ij + T_ji - T_ii - T_jj + c_ij."""
    n = len(perm)
    F, D, p = _mat(F, n), _mat(D, n), _vec(perm, n)
    out = np.zeros(n * (n - 1) // 2, dtype=np.int64)
    _load().orc_delta_table_contraction(n, _p32(F), _p32(D), _p32(p), _p64(out))
    return out


def delta_update(F, D, perm_before, r, s, table) -> np.ndarray:
    """Incremental update of a packed delta table after applying (r, s) to perm_before."""
    n = len(perm_before)
    F, D, p = _mat(F, n), _mat(D, n), _vec(perm_before, n)
    tab = np.array(table, dtype=np.int64, copy=True)
    _load().orc_delta_update(n, _p32(F), _p32(D), _p32(p), int(r), int(s), _p64(tab))
    return tab


def philox(counter, key) -> np.ndarray:
    """Philox4x64-10 block for a 4-word counter and 2-word key (uint64)."""
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    _load().orc_philox4x64_10(c.ctypes.data_as(_u64p), k.ctypes.data_as(_u64p), out.ctypes.data_as(_u64p))
    return out


def tenure(seed, it, start, lo, hi) -> int:
    return int(_load().orc_tenure(int(seed), int(it), int(start), int(lo), int(hi)))


def two_opt(F, D, perm, max_iters=0, mode=1, trace_cap=0):
    """Best-improvement 2opt to a local optimum.  Returns (perm, cost, steps, trace)."""
    n = len(perm)
    F, D = _mat(F, n), _mat(D, n)
    p = np.array(perm, dtype=np.int32, copy=True)
    c = np.zeros(1, dtype=np.int64)
    st = np.zeros(1, dtype=np.int32)
    tr = np.zeros(max(trace_cap, 1) * 4, dtype=np.int64)
    rc = _load().orc_2opt(n, _p32(F), _p32(D), _p32(p), int(max_iters), int(mode), _p64(c), _p32(st),
                          _p64(tr) if trace_cap else None, int(trace_cap))
    if rc != 0:
        raise MemoryError("oracle 2opt: out of memory")
    steps = int(st[0])
    return p, int(c[0]), steps, tr[:4 * min(steps, trace_cap)].reshape(-1, 4)


def tabu(F, D, perm, iters, lo, hi, seed, start=0, mode=1, trace_cap=0):
    """Tabu search.  Returns (best_perm, best_cost, iters_done, trace)."""
    n = len(perm)
    F, D, p0 = _mat(F, n), _mat(D, n), _vec(perm, n)
    bp = np.zeros(n, dtype=np.int32)
    bc = np.zeros(1, dtype=np.int64)
    done = np.zeros(1, dtype=np.int32)
    tr = np.zeros(max(trace_cap, 1) * 4, dtype=np.int64)
    rc = _load().orc_tabu(n, _p32(F), _p32(D), _p32(p0), int(iters), int(lo), int(hi),
                          int(seed), int(start), int(mode), _p32(bp), _p64(bc), _p32(done),
                          _p64(tr) if trace_cap else None, int(trace_cap))
    if rc != 0:
        raise MemoryError("oracle tabu: out of memory")
    d = int(done[0])
    return bp, int(bc[0]), d, tr[:4 * min(d, trace_cap)].reshape(-1, 4)


def tabu_freq(F, D, perm, iters, lo, hi, seed, start=0, div=0, trace_cap=0, attr=0):
    """Tabu search keeping the frequency memory, with the frequency-based diversification
    move every time the best cost has not improved for more than div iterations (div = 0:
    none); attr 0 makes pairs of locations tabu, 1 the units just moved, 2 the return of
    both units to locations they just left.  Returns (best_perm, best_cost, iters_done,
    freq, trace)."""
    n = len(perm)
    F, D, p0 = _mat(F, n), _mat(D, n), _vec(perm, n)
    m = n * (n - 1) // 2
    bp = np.zeros(n, dtype=np.int32)
    bc = np.zeros(1, dtype=np.int64)
    done = np.zeros(1, dtype=np.int32)
    freq = np.zeros(max(m, 1), dtype=np.int32)
    tr = np.zeros(max(trace_cap, 1) * 4, dtype=np.int64)
    rc = _load().orc_tabu_freq(n, _p32(F), _p32(D), _p32(p0), int(iters), int(lo), int(hi), int(seed),
                               int(start), int(div), int(attr), _p32(bp), _p64(bc), _p32(done), _p32(freq),
                               _p64(tr) if trace_cap else None, int(trace_cap))
    if rc != 0:
        raise MemoryError("oracle tabu_freq: out of memory")
    d = int(done[0])
    return bp, int(bc[0]), d, freq[:m], tr[:4 * min(d, trace_cap)].reshape(-1, 4)
