"""GPU tests of the continuous-batching tabu server.

Each request's result must be the same when it runs alone in one go (qap_tabu, start
id 0), when it runs in a mix of other requests of uneven n and is cut into many chunks,
and, for a sample, what the oracle gives.  Admission is bounded by the memory pool: with
a pool that holds only a few requests, the rest wait in the queue and still finish with
the same results.
"""
import sys

import numpy as np
import pytest

import oracle
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


def requests(seed, sizes, itmin, itmax):
    rng = np.random.default_rng(seed)
    out = []
    for t, n in enumerate(sizes):
        sp = float(rng.uniform(0.0, 0.8))
        F = W.sparse_matrix(rng, n, sp, 0, 99)
        D = W.uniform_matrix(rng, n, 0, 99)
        if t % 4 == 3:   # some symmetric instances
            F = np.triu(F) + np.triu(F, 1).T
            D = np.triu(D) + np.triu(D, 1).T
            np.fill_diagonal(D, 0)
        it = int(rng.integers(itmin, itmax + 1))
        lo, hi = W.tabu_tenure_range(n)
        seed_r = int(rng.integers(0, 2**62))
        out.append((F.astype(np.int32), D.astype(np.int32), W.starts(rng, n, 1)[0], it, lo, hi, seed_r))
    return out


def alone(req):
    F, D, p, it, lo, hi, seed = req
    with qap.Handle(F, D) as h:
        bp, bc, bd = h.tabu(p[None, :], it, lo, hi, seed)
    return bp[0], int(bc[0]), int(bd[0])


def serve_all(reqs, pool_bytes=1 << 28, max_active=64, chunk_ms=0.2, limit_steps=100000):
    res = {}
    peak_running, saw_queue = 0, False
    with qap.Server(pool_bytes, max_active, chunk_ms) as s:
        tickets = [s.submit(*r) for r in reqs]
        steps = 0
        while len(res) < len(reqs):
            f, running, queued = s.step()
            peak_running = max(peak_running, running + f)
            saw_queue = saw_queue or queued > 0
            for t in tickets:
                if t not in res:
                    r = s.result(t)
                    if r is not None:
                        res[t] = r
            steps += 1
            assert steps < limit_steps, "server made no progress"
        stats = s.stats()
        assert stats["running"] == 0 and stats["queued"] == 0 and stats["pool_used"] == 0
    return [res[t] for t in tickets], peak_running, saw_queue, stats


def test_serve_results_equal_alone_and_oracle():
    reqs = requests(51, [30, 47, 64, 90, 31, 128, 150, 77, 100, 64, 33, 176], 300, 2500)
    note("serve mix of %d requests, chunk 0.2 ms" % len(reqs))
    got, peak, _, stats = serve_all(reqs)
    assert stats["chunks"] > len(reqs)   # searches were cut into several chunks
    for i, r in enumerate(reqs):
        ep, ec, ed = alone(r)
        assert (got[i][0] == ep).all() and got[i][1] == ec and got[i][2] == ed, i
    for i in (0, 2, 6):
        F, D, p, it, lo, hi, seed = reqs[i]
        bp, bc, done, _ = oracle.tabu(F, D, p, it, lo, hi, seed, 0)
        assert (got[i][0] == bp).all() and got[i][1] == bc and got[i][2] == done, i


def test_serve_admission_bounded_by_pool():
    reqs = requests(52, [40, 60, 80, 100, 120, 60, 40], 200, 800)
    with qap.Server(1 << 20, 1, 1.0) as probe:
        pool = 2 * probe.footprint(120) + 4096
    note("serve with a pool of %d bytes" % pool)
    got, peak, saw_queue, _ = serve_all(reqs, pool_bytes=pool, chunk_ms=0.1)
    assert saw_queue and peak < len(reqs)
    for i, r in enumerate(reqs):
        ep, ec, ed = alone(r)
        assert (got[i][0] == ep).all() and got[i][1] == ec and got[i][2] == ed, i


def test_serve_rejects_what_cannot_run():
    rng = np.random.default_rng(9)
    F, D = W.random_instance(rng, 40, 0, 99)
    with qap.Server(1 << 20, 1, 1.0) as probe:
        need = probe.footprint(40)
    with qap.Server(need - 1024, 4, 1.0) as s:
        with pytest.raises(qap.QapError) as ei:
            s.submit(F, D, np.arange(40), 100, 3, 5, 1)
        assert ei.value.code == qap.QAP_E_NOMEM
    with qap.Server(1 << 24, 4, 1.0) as s:
        bad = np.arange(40)
        bad[0] = 1
        with pytest.raises(qap.QapError) as ei:
            s.submit(F, D, bad, 100, 3, 5, 1)
        assert ei.value.code == qap.QAP_E_NOT_PERM
        G = F.copy()
        G[0, 1] = 300
        with pytest.raises(qap.QapError) as ei:
            s.submit(G, D, np.arange(40), 100, 3, 5, 1)
        assert ei.value.code == qap.QAP_E_RANGE
        t = s.submit(F, D, np.arange(40), 0, 3, 5, 1)   # zero iterations: the start itself
        for _ in range(10):
            s.step()
            r = s.result(t)
            if r is not None:
                break
        assert r is not None and (r[0] == np.arange(40)).all() and r[2] == 0


def test_serve_chunked_equals_unchunked():
    reqs = requests(53, [64, 100], 3000, 3000)
    note("serve chunked vs one chunk")
    a, _, _, sa = serve_all(reqs, chunk_ms=0.05)
    b, _, _, sb = serve_all(reqs, chunk_ms=0.0)
    assert sa["chunks"] > sb["chunks"] == 2
    for x, y in zip(a, b):
        assert (x[0] == y[0]).all() and x[1:3] == y[1:3]


def test_serve_admission_bounded_by_slots():
    reqs = requests(54, [50, 70, 90, 110, 60, 80], 300, 900)
    note("serve with two slots")
    got, peak, saw_queue, stats = serve_all(reqs, max_active=2, chunk_ms=0.1)
    assert saw_queue and peak <= 2
    for i, r in enumerate(reqs):
        ep, ec, ed = alone(r)
        assert (got[i][0] == ep).all() and got[i][1] == ec and got[i][2] == ed, i


def test_serve_c5_stream_head_equals_oracle():
    """The first 48 requests of the serving stream (n from 30 to 256, 2000 to 20 000
    iterations, F sparsity up to 80%), all submitted at once to a server with 2 ms chunks;
    every result is recomputed by the oracle (start id 0)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    stream = W.c5_stream(count=48)
    reqs = []
    for r in stream:
        lo, hi = W.tabu_tenure_range(r.inst.n)
        reqs.append((r.inst.F, r.inst.D, r.inst.perms[0], r.iters, lo, hi, r.inst.seed))
    note("serve the first %d requests of the serving stream, chunk 2 ms" % len(reqs))
    got, _, _, stats = serve_all(reqs, pool_bytes=1 << 30, max_active=256, chunk_ms=2.0)
    assert stats["chunks"] >= len(reqs)

    def one(r):
        F, D, p, it, lo, hi, seed = r
        return oracle.tabu(F, D, p, it, lo, hi, seed, 0)

    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as ex:
        want = list(ex.map(one, reqs))
    for i, (g, e) in enumerate(zip(got, want)):
        assert (g[0] == e[0]).all() and g[1] == e[1] and g[2] == e[2], (i, reqs[i][0].shape[0])
