"""GPU parity of the wide streamed kernel, which serves 256 < n <= 512.

Beyond n = 256 the permuted flows G = F[p][p] and G^T no longer fit in LDS beside the
rest of a search, so the wide kernel keeps them, like D and D^T, in global scratch (the
move exchanges two of their rows and columns in place, between the workgroup barriers),
runs up to four (index, family) tasks per lane, and the
starting neighbourhood comes from the blocked matrix-core table kernel.  Tabu searches
without the frequency memory keep a compact tabu state (a bit per slot in LDS and a ring
of recent moves) while the tenures fit the ring, and the per-slot tenure words beyond
that.  Every case is compared bit for bit with the oracle (the frequency memory and tabu
attributes on this kernel are covered with the other tile shapes).
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


def test_wide_table_row_that_is_no_permutation_is_zero():
    """The blocked matrix-core table above n = 256: a start that is not a permutation gets
    a zero row (every block of the start clears its own entries), the others are exact."""
    import torch
    n = 300
    rng = np.random.default_rng(9150)
    F, D = W.random_instance(rng, n, 0, 255, diag=True)
    perms = W.starts(rng, n, 3)
    bad = perms.copy()
    bad[1, 5] = bad[1, 6]
    note("wide table with a bad row n=300")
    with qap.Handle(F, D) as h:
        dp = torch.from_numpy(bad).cuda()
        dt = torch.full((3, n * (n - 1) // 2), 7, dtype=torch.int32, device="cuda")
        h.delta_table_async(dp, dt)
        torch.cuda.synchronize()
        t = dt.cpu().numpy()
    assert (t[1] == 0).all()
    for j in (0, 2):
        assert (t[j] == oracle.delta_table(F, D, bad[j])).all(), j


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


def test_wide_register_tiles_say_so():
    n = 300
    rng = np.random.default_rng(9400)
    F, D = W.random_instance(rng, n, 0, 99)
    note("wide register-tile rejections n=300")
    with qap.Handle(F, D) as h:
        for rows in (1, 2, 4, 8, 16):
            with pytest.raises(qap.QapError) as ei:
                h.set_tile_rows("tabu", rows)
            assert ei.value.code == qap.QAP_E_UNSUPPORTED


def test_wide_in_a_batch_equals_the_oracle():
    """Instances above n = 256 (the wide streamed form, G in the plan's scratch, their
    starting tables by Eq. (2)) beside register-tile and streamed ones in one batch, run
    twice from a captured-graph-free plan: every start equals oracle.tabu."""
    sizes, ks, iters = [300, 40, 384, 200, 257], [2, 2, 1, 1, 1], 120
    rng = np.random.default_rng(9410)
    insts, lohi, seeds = [], [], []
    for t, n in enumerate(sizes):
        F, D = W.random_instance(rng, n, 0, 99, symmetric=(t == 2))
        insts.append((F, D, W.starts(rng, n, ks[t])))
        lohi.append(W.paper_tenure_range(n))
        seeds.append(int(rng.integers(0, 2**62)))
    note("wide batch sizes=%s k=%s iters=%d" % (sizes, ks, iters))
    hs = [qap.Handle(F, D) for F, D, _ in insts]
    perms = np.concatenate([P.reshape(-1) for _, _, P in insts]).astype(np.int32)
    p, c, d = qap.tabu_batch(hs, perms, ks, iters, [a for a, _ in lohi], [b for _, b in lohi], seeds)
    jobs = [(i, j) for i in range(len(sizes)) for j in range(ks[i])]
    res = pmap(lambda a: oracle.tabu(insts[a[0]][0], insts[a[0]][1], insts[a[0]][2][a[1]], iters,
                                     lohi[a[0]][0], lohi[a[0]][1], seeds[a[0]], a[1]), jobs)
    off = 0
    for t, ((i, j), r) in enumerate(zip(jobs, res)):
        n = sizes[i]
        assert (p[off:off + n] == r[0]).all() and c[t] == r[1] and d[t] == r[2], (i, j)
        off += n
    for h in hs:
        h.close()


def test_wide_in_the_server_equals_the_oracle():
    """Requests above n = 256 served in chunks beside smaller ones (a launch of the wide
    resume kernel of their own each step): every result equals oracle.tabu."""
    sizes, iters = [300, 60, 260, 180], [160, 400, 120, 200]
    rng = np.random.default_rng(9420)
    reqs = []
    for n, it in zip(sizes, iters):
        F, D = W.random_instance(rng, n, 0, 99)
        reqs.append((F, D, W.starts(rng, n, 1)[0], it, W.tabu_tenure_range(n), int(rng.integers(0, 2**62))))
    note("wide server sizes=%s iters=%s" % (sizes, iters))
    with qap.Server(1 << 28, 8, 0.3) as s:
        tickets = [s.submit(F, D, p0, it, lo, hi, seed) for F, D, p0, it, (lo, hi), seed in reqs]
        out = {}
        for _ in range(10000):
            s.step()
            for t in tickets:
                if t not in out:
                    r = s.poll(t)
                    if r is not None:
                        out[t] = r
            if len(out) == len(tickets):
                break
        assert len(out) == len(tickets)
        assert s.stats()["steps"] > 1   # chunked
    res = pmap(lambda q: oracle.tabu(q[0], q[1], q[2], q[3], q[4][0], q[4][1], q[5], 0), reqs)
    for t, r in zip(tickets, res):
        assert (out[t][0] == r[0]).all() and out[t][1] == r[1], t


@pytest.mark.parametrize("sym", [False, True])
def test_wide_short_tenure_past_the_tenure_ring(sym):
    """n = 512 with the paper's short tenure and more iterations than the 512-entry tenure
    ring holds, so tabu expiry, aspiration against expired moves and the ring refill all
    run on the wide kernel, against oracle.tabu."""
    n, k, iters = 512, 2, 700
    rng = np.random.default_rng(9430 + sym)
    F, D = W.random_instance(rng, n, 0, 99, symmetric=sym)
    perms = W.starts(rng, n, k)
    lo, hi = W.paper_tenure_range(n)
    note("wide short tenure n=512 sym=%d iters=%d" % (sym, iters))
    with qap.Handle(F, D) as h:
        p, c, d = h.tabu(perms, iters, lo, hi, 21)
    res = pmap(lambda j: oracle.tabu(F, D, perms[j], iters, lo, hi, 21, j), range(k))
    for j, r in enumerate(res):
        assert (p[j] == r[0]).all() and c[j] == r[1] and d[j] == r[2], j


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


@pytest.mark.parametrize("sym,lo,hi", [(False, 0, 2), (True, 1, 3), (False, 5, 40)])
def test_wide_compact_tabu_state_short_tenures(sym, lo, hi):
    """Tenures of 0 and 1 (the move is admissible again at once), pairs made tabu again
    before they expire, and many expiries an iteration: the compact tabu state of the
    wide kernel against oracle.tabu."""
    n, k, iters = 300, 3, 400
    rng = np.random.default_rng(9500 + lo + hi)
    F, D = W.random_instance(rng, n, 0, 99, symmetric=sym)
    perms = W.starts(rng, n, k)
    note("wide compact tabu n=%d sym=%d tenure [%d, %d] iters=%d" % (n, sym, lo, hi, iters))
    with qap.Handle(F, D) as h:
        p, c, d = h.tabu(perms, iters, lo, hi, 31)
    res = pmap(lambda j: oracle.tabu(F, D, perms[j], iters, lo, hi, 31, j), range(k))
    for j, r in enumerate(res):
        assert (p[j] == r[0]).all() and c[j] == r[1] and d[j] == r[2], j


def test_wide_tenures_past_the_compact_ring():
    """Tenures of 1024 and more do not fit the compact state's ring of moves: such searches
    keep a tenure word per slot, against oracle.tabu."""
    n, k, iters, lo, hi = 260, 2, 120, 1020, 1100
    rng = np.random.default_rng(9600)
    F, D = W.random_instance(rng, n, 0, 99)
    perms = W.starts(rng, n, k)
    note("wide per-slot tenure words n=%d tenure [%d, %d]" % (n, lo, hi))
    with qap.Handle(F, D) as h:
        p, c, d = h.tabu(perms, iters, lo, hi, 41)
    res = pmap(lambda j: oracle.tabu(F, D, perms[j], iters, lo, hi, 41, j), range(k))
    for j, r in enumerate(res):
        assert (p[j] == r[0]).all() and c[j] == r[1] and d[j] == r[2], j
