"""CPU-side checks of the C ABI: the library loads, exports every symbol include/qap.h
declares, maps error codes to text, and rejects invalid arguments before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2307_11248_amd import qap

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "qap.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qap_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_binding_exports():
    assert header_functions() == sorted(qap.EXPORTS)


def test_library_exports_every_header_symbol():
    lib = ctypes.CDLL(qap.LIB_PATH)
    for name in header_functions():
        assert hasattr(lib, name), name


def test_strerror_codes():
    L = qap.lib()
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert L.qap_strerror(code)
    assert L.qap_strerror(-99) == b"unknown error"


def _create(F, D, n):
    L = qap.lib()
    h = ctypes.c_void_p()
    Fa = np.ascontiguousarray(F, dtype=np.int32)
    Da = np.ascontiguousarray(D, dtype=np.int32)
    return L.qap_create(Fa.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                        Da.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n, ctypes.byref(h))


def test_create_rejects_out_of_range_entries():
    F = np.zeros((5, 5), dtype=np.int32)
    D = np.zeros((5, 5), dtype=np.int32)
    F[1, 2] = 256
    assert _create(F, D, 5) == qap.QAP_E_RANGE
    F[1, 2] = -1
    assert _create(F, D, 5) == qap.QAP_E_RANGE


def test_create_rejects_bad_sizes():
    z = np.zeros((1, 1), dtype=np.int32)
    assert _create(z, z, 1) == qap.QAP_E_INVALID
    assert _create(z, z, qap.QAP_NMAX + 1) == qap.QAP_E_INVALID


def test_null_handle_calls():
    L = qap.lib()
    assert L.qap_destroy(None) == 0
    assert L.qap_size(None) == qap.QAP_E_INVALID
    assert L.qap_set_tile_rows(None, 0, 4) == qap.QAP_E_INVALID


def test_binding_size_limits_match_the_header():
    txt = open(os.path.join(ROOT, "include", "qap.h")).read()
    defs = dict(re.findall(r"#define (QAP_NMAX\w*) (\d+)", txt))
    assert int(defs["QAP_NMAX"]) == qap.QAP_NMAX == 512
    assert int(defs["QAP_NMAX_BATCH"]) == qap.QAP_NMAX_BATCH == 512


def test_noalloc_scratch_size_matches_the_header():
    txt = open(os.path.join(ROOT, "include", "qap.h")).read()
    m = re.search(r"#define QAP_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", txt)
    assert m and int(m.group(1)) << int(m.group(2)) == qap.QAP_NOALLOC_SCRATCH_BYTES


def test_noalloc_rejects_bad_arguments():
    L = qap.lib()
    assert L.qap_tabu_noalloc_async(None, None, 1, 10, 1, 2, 0, 0, None, None, None) == qap.QAP_E_INVALID
