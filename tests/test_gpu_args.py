"""Argument checks of the C ABI that need a live handle: tabu runs whose tabu-until
iteration (it + t, Sec. 4.3) would not fit int32 are rejected by every tabu entry point,
and the edge just inside the bound is accepted."""
import ctypes

import numpy as np
import pytest

from paper_2307_11248_amd import qap
from paper_2307_11248_amd import workloads as W

pytestmark = pytest.mark.gpu

I32MAX = 2**31 - 1


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.init()
    yield


def _i32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _i64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def test_tabu_until_overflow_rejected_everywhere():
    rng = np.random.default_rng(1)
    n, k = 9, 2
    F, D = (np.ascontiguousarray(x, dtype=np.int32) for x in W.random_instance(rng, n, 0, 99))
    perms = np.ascontiguousarray(W.starts(rng, n, k), dtype=np.int32)
    L = qap.lib()
    bad = [(10, 0, I32MAX), (I32MAX - 5, 3, 10), (5, I32MAX - 1, I32MAX)]
    with qap.Handle(F, D) as h:
        for iters, lo, hi in bad:
            p = perms.copy()
            best = np.zeros(k, dtype=np.int64)
            assert L.qap_tabu(h.ptr, _i32(p), k, iters, lo, hi, 1, _i64(best), None) == qap.QAP_E_INVALID
            m = 1
            hs = (ctypes.c_void_p * 1)(h.ptr)
            ks = np.array([k], dtype=np.int32)
            los, his = np.array([lo], dtype=np.int32), np.array([hi], dtype=np.int32)
            seeds = np.array([1], dtype=np.uint64)
            b = ctypes.c_void_p()
            assert L.qap_batch_create(hs, m, _i32(ks), iters, _i32(los), _i32(his),
                                      seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), None,
                                      ctypes.byref(b)) == qap.QAP_E_INVALID
        # just inside: iters + hi = INT32_MAX - 1 with no iterations to run
        p = perms.copy()
        best = np.zeros(k, dtype=np.int64)
        done = np.zeros(k, dtype=np.int32)
        assert L.qap_tabu(h.ptr, _i32(p), k, 0, 0, I32MAX - 1, 1, _i64(best), _i32(done)) == 0
        assert (p == perms).all() and (done == 0).all() and (best == h.cost(perms)).all()
    with qap.Server(1 << 26, 4, 1.0) as srv, qap.Handle(F, D) as h:
        t = ctypes.c_int64()
        for iters, lo, hi in bad:
            assert L.qap_server_submit_matrices(srv._s, _i32(F), _i32(D), n, _i32(perms[0]), iters, lo, hi, 1,
                                                ctypes.byref(t)) == qap.QAP_E_INVALID
            assert L.qap_server_submit(srv._s, h.ptr, _i32(perms[0]), iters, lo, hi, 1,
                                       ctypes.byref(t)) == qap.QAP_E_INVALID
