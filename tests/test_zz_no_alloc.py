"""The tabu entry point that allocates nothing (qap_tabu_noalloc_async) against the one
that does (qap_tabu_async), through the C ABI: same starts, same arguments, identical
best permutations, costs and move counts.  Two calls in a row on the shared fixed
scratch, the second with a smaller input, on each kernel family that uses scratch: the
register-tile kernels (neighbourhood tables only), the streamed kernel (tables and tile
state) and the wide streamed kernel (tables, tile state and G, G^T).  A call that needs
more than the fixed scratch is refused with QAP_E_SCRATCH and changes nothing.
"""
import sys

import numpy as np
import pytest

from paper_2307_11248_amd import qap
from paper_2307_11248_amd import workloads as W

pytestmark = pytest.mark.gpu


def note(msg):
    sys.__stderr__.write("[gpu-case] %s\n" % msg)
    sys.__stderr__.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.init()
    yield


def run_pair(h, perms, iters, lo, hi, seed, start_base=0):
    """(perm, best, done) from qap_tabu_async and from qap_tabu_noalloc_async."""
    import torch
    out = []
    for noalloc in (False, True):
        dp = torch.from_numpy(perms).cuda()
        db = torch.zeros(perms.shape[0], dtype=torch.int64, device="cuda")
        dd = torch.zeros(perms.shape[0], dtype=torch.int32, device="cuda")
        f = h.tabu_noalloc_async if noalloc else h.tabu_async
        f(dp, iters, lo, hi, seed, db, dd, start_base=start_base)
        torch.cuda.synchronize()
        out.append((dp.cpu().numpy(), db.cpu().numpy(), dd.cpu().numpy()))
    return out


def check_same(a, b, what):
    assert (a[0] == b[0]).all(), what + ": permutations differ"
    assert (a[1] == b[1]).all(), what + ": costs differ"
    assert (a[2] == b[2]).all(), what + ": moves differ"


# (n, k, iters, symmetric, forced tile rows or None): first a larger call, then a smaller
CASES = [
    ("register tiles", [(96, 64, 400, False, None), (40, 8, 300, True, None)]),
    ("streamed", [(200, 6, 150, False, -8), (180, 3, 120, True, -8)]),
    ("wide streamed", [(384, 4, 60, False, None), (300, 2, 50, True, None)]),
]


@pytest.mark.parametrize("name,calls", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_tabu_async(name, calls):
    for i, (n, k, iters, sym, rows) in enumerate(calls):
        note("noalloc %s call %d: n=%d k=%d iters=%d sym=%d" % (name, i, n, k, iters, sym))
        rng = np.random.default_rng(9000 + 17 * n + i)
        F, D = W.random_instance(rng, n, 0, 99, symmetric=sym)
        perms = W.starts(rng, n, k)
        lo, hi = W.tabu_tenure_range(n)
        with qap.Handle(F, D) as h:
            if rows is not None:
                h.set_tile_rows("tabu", rows)
            a, b = run_pair(h, perms, iters, lo, hi, seed=77 + i, start_base=5 * i)
        check_same(a, b, "%s call %d" % (name, i))
        assert (b[2] == iters).all()


def test_noalloc_refuses_calls_beyond_its_scratch():
    import torch
    n = 256
    m = n * (n - 1) // 2
    k = qap.QAP_NOALLOC_SCRATCH_BYTES // (4 * m) + 1   # the tables alone overflow it
    note("noalloc overflow: n=%d k=%d" % (n, k))
    rng = np.random.default_rng(4242)
    F, D = W.random_instance(rng, n, 0, 99)
    with qap.Handle(F, D) as h:
        perms = np.tile(np.arange(n, dtype=np.int32), (k, 1))
        dp = torch.from_numpy(perms).cuda()
        db = torch.full((k,), -7, dtype=torch.int64, device="cuda")
        with pytest.raises(qap.QapError) as ei:
            h.tabu_noalloc_async(dp, 10, 1, 5, 1, db)
        assert ei.value.code == qap.QAP_E_SCRATCH
        torch.cuda.synchronize()
        assert (db.cpu().numpy() == -7).all()
        assert (dp.cpu().numpy() == perms).all()
