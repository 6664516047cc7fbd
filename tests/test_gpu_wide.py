"""GPU parity of the wide streamed kernel, which serves 256 < n <= 512.

Beyond n = 256 the permuted flows G = F[p][p] and G^T no longer fit in LDS beside the
rest of a search, so the wide kernel keeps them, like D and D^T, in global scratch (the
move exchanges two of their rows and columns in place, between the workgroup barriers),
runs up to four (index, family) tasks per lane, and the
starting neighbourhood is evaluated entry by entry from Eq. (2).  Every case is compared
bit for bit with the oracle (the frequency memory and tabu attributes on this kernel are
covered with the other tile shapes).  The batched and served paths stop at n = 256 and
say so.
"""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2307_11248_amd import qap
from paper_2307_11248_amd import workloads as W

pytestmark = pytest.mark.gpu

WORKERS = max(1, min(16, os.cpu_count() or 1))


def note(msg):
    sys.__stderr__.write("[gpu-case] %s\n" % msg)
    sys.__stderr__.flush()


def pmap(f, items):
    with ThreadPoolExecutor(WORKERS) as ex:
        return list(ex.map(f, items))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.init()
    yield


@pytest.mark.parametrize("n,sym", [(257, False), (300, True), (512, False), (512, True)])
def test_wide_cost_and_neighbourhood_equal_the_oracle(n, sym):
    """Eq. (1) costs and the Eq. (2) neighbourhood of three starts, every entry."""
    rng = np.random.default_rng(9100 + n + sym)
    F, D = W.random_instance(rng, n, 0, 255, symmetric=sym, diag=True)
    perms = W.starts(rng, n, 3)
    note("wide cost and table n=%d sym=%s" % (n, sym))
    with qap.Handle(F, D) as h:
        c = h.cost(perms)
        t = h.delta_table(perms)
    for j in range(3):
        assert c[j] == oracle.cost(F, D, perms[j]), j
        assert (t[j] == oracle.delta_table(F, D, perms[j])).all(), j


@pytest.mark.parametrize("n,sym,diag", [(257, False, False), (300, True, False), (384, False, True),
                                        (451, True, True), (512, False, False)])
def test_wide_tabu_and_two_opt_equal_the_oracle(n, sym, diag):
    rng = np.random.default_rng(9200 + n)
    F, D = W.random_instance(rng, n, 0, 99, symmetric=sym, diag=diag)
    perms = W.starts(rng, n, 3)
    lo, hi = W.tabu_tenure_range(n)
    iters = 200
    note("wide tabu and 2opt n=%d sym=%s" % (n, sym))
    with qap.Handle(F, D) as h:
        assert h.tile_rows("tabu")[0] == -8 and h.tile_rows("2opt")[0] == -8
        p, c, d = h.tabu(perms, iters, lo, hi, 321)
        q, qc, qs = h.two_opt(perms, max_iters=50)
    res = pmap(lambda j: oracle.tabu(F, D, perms[j], iters, lo, hi, 321, j), range(3))
    for j, r in enumerate(res):
        assert (p[j] == r[0]).all() and c[j] == r[1] and d[j] == r[2], j
    res = pmap(lambda j: oracle.two_opt(F, D, perms[j], max_iters=50), range(3))
    for j, r in enumerate(res):
        assert (q[j] == r[0]).all() and qc[j] == r[1] and qs[j] == r[2], j


def test_wide_extreme_entries_and_plain_launches():
    """Entries at 0 and 255 (the largest deltas n = 512 allows), and the one-launch-per-
    start form against the batched launch of the same starts."""
    import torch
    n = 512
    rng = np.random.default_rng(9300)
    F = (rng.random((n, n)) < 0.5).astype(np.int32) * 255
    D = (rng.random((n, n)) < 0.5).astype(np.int32) * 255
    perms = W.starts(rng, n, 2)
    lo, hi = W.tabu_tenure_range(n)
    iters = 120
    note("wide extreme entries n=512")
    with qap.Handle(F, D) as h:
        p, c, d = h.tabu(perms, iters, lo, hi, 9)
        dp = torch.from_numpy(perms).cuda()
        db = torch.zeros(2, dtype=torch.int64, device="cuda")
        dd = torch.zeros(2, dtype=torch.int32, device="cuda")
        h.tabu_async(dp, iters, lo, hi, 9, db, dd, plain=True)
        torch.cuda.synchronize()
        assert (dp.cpu().numpy() == p).all() and (db.cpu().numpy() == c).all() and (dd.cpu().numpy() == d).all()
    res = pmap(lambda j: oracle.tabu(F, D, perms[j], iters, lo, hi, 9, j), range(2))
    for j, r in enumerate(res):
        assert (p[j] == r[0]).all() and c[j] == r[1] and d[j] == r[2], j


def test_wide_paths_that_stop_at_256_say_so():
    n = 300
    rng = np.random.default_rng(9400)
    F, D = W.random_instance(rng, n, 0, 99)
    perms = W.starts(rng, n, 1)
    note("wide rejections n=300")
    with qap.Handle(F, D) as h:
        for rows in (1, 2, 4, 8, 16):
            with pytest.raises(qap.QapError) as ei:
                h.set_tile_rows("tabu", rows)
            assert ei.value.code == qap.QAP_E_UNSUPPORTED
        with pytest.raises(qap.QapError) as ei:
            qap.tabu_batch([h], perms.reshape(-1), [1], 10, [30], [90], [1])
        assert ei.value.code == qap.QAP_E_UNSUPPORTED
    with qap.Server(1 << 26, 4, 0.1) as s:
        with pytest.raises(qap.QapError) as ei:
            s.footprint(n)
        assert ei.value.code == qap.QAP_E_UNSUPPORTED


def test_wide_table_taking_entry_points_and_full_descent():
    """The search kernels alone on a table built by qap_delta_table_async (the bench's
    step), against the entry points that build their own; and 2opt run to the local
    optimum (no move cap) against the oracle."""
    import torch
    n = 300
    rng = np.random.default_rng(9500)
    F, D = W.random_instance(rng, n, 0, 99, symmetric=True)
    perms = W.starts(rng, n, 2)
    lo, hi = W.tabu_tenure_range(n)
    iters = 150
    note("wide table-taking entry points n=300")
    with qap.Handle(F, D) as h:
        p, c, d = h.tabu(perms, iters, lo, hi, 17)
        q, qc, qs = h.two_opt(perms)
        m = n * (n - 1) // 2
        dp = torch.from_numpy(perms).cuda()
        dt = torch.empty((2, m), dtype=torch.int32, device="cuda")
        db = torch.zeros(2, dtype=torch.int64, device="cuda")
        dd = torch.zeros(2, dtype=torch.int32, device="cuda")
        h.delta_table_async(dp, dt)
        h.tabu_with_table_async(dp, dt, iters, lo, hi, 17, db, dd)
        torch.cuda.synchronize()
        assert (dp.cpu().numpy() == p).all() and (db.cpu().numpy() == c).all() and (dd.cpu().numpy() == d).all()
        dp2 = torch.from_numpy(perms).cuda()
        h.delta_table_async(dp2, dt)
        h.two_opt_with_table_async(dp2, dt, db, dd)
        torch.cuda.synchronize()
        assert (dp2.cpu().numpy() == q).all() and (db.cpu().numpy() == qc).all() and (dd.cpu().numpy() == qs).all()
    res = pmap(lambda j: oracle.two_opt(F, D, perms[j]), range(2))
    for j, r in enumerate(res):
        assert (q[j] == r[0]).all() and qc[j] == r[1] and qs[j] == r[2], j
