"""GPU tests of the server's request interface: submissions on existing handles, polling,
the queue limit, cancellation, a failure of one search that leaves the others serving,
admission past a request that does not fit, and the server's own stepping thread.  Every
result that is returned must equal the same request run alone (qap_tabu, start id 0), and
a sample is checked against the oracle."""
import sys
import time

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


def make_reqs(seed, sizes, itmin, itmax):
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        F = W.sparse_matrix(rng, n, float(rng.uniform(0.0, 0.8)), 0, 99)
        D = W.uniform_matrix(rng, n, 0, 99)
        it = int(rng.integers(itmin, itmax + 1))
        lo, hi = W.tabu_tenure_range(n)
        out.append((F, D, W.starts(rng, n, 1)[0], it, lo, hi, int(rng.integers(0, 2**62))))
    return out


def alone(req):
    F, D, p, it, lo, hi, seed = req
    with qap.Handle(F, D) as h:
        bp, bc, bd = h.tabu(p[None, :], it, lo, hi, seed)
    return bp[0], int(bc[0]), int(bd[0])


def drive(s, tickets, done, limit=200000):
    steps = 0
    while any(t not in done for t in tickets):
        s.step()
        for t in tickets:
            if t not in done:
                r = s.result(t)
                if r is not None:
                    done[t] = r
        steps += 1
        assert steps < limit, "server made no progress"


def test_submit_on_handles_and_poll():
    note("serve: submit on handles, poll")
    reqs = make_reqs(10, [24, 57, 90, 131, 180, 40], 300, 1500)
    hs = [qap.Handle(F, D) for F, D, *_ in reqs]
    try:
        with qap.Server(1 << 27, 8, 0.1) as s:
            tickets = [s.submit_handle(h, r[2], *r[3:]) for h, r in zip(hs, reqs)]
            got = {}
            for _ in range(200000):
                s.step()
                for t in tickets:
                    if t not in got:
                        r = s.poll(t)
                        if r is not None:
                            got[t] = r
                if len(got) == len(tickets):
                    break
            assert len(got) == len(tickets)
            st = s.stats()
            assert st["finished"] == len(reqs) and st["pool_used"] == 0
        for t, r in zip(tickets, reqs):
            bp, bc, _ = alone(r)
            assert (got[t][0] == bp).all() and got[t][1] == bc
        # the oracle on two of them
        for i in (0, 5):
            F, D, p, it, lo, hi, seed = reqs[i]
            obp, obc, _, _ = oracle.tabu(F, D, p, it, lo, hi, seed, 0)
            assert (got[tickets[i]][0] == obp).all() and got[tickets[i]][1] == obc
    finally:
        for h in hs:
            h.close()


def test_queue_limit_busy():
    note("serve: queue limit")
    reqs = make_reqs(11, [20, 21, 22], 50, 60)
    with qap.Server(1 << 26, 4, 0.1) as s:
        s.set_queue_limit(2)
        t0 = s.submit(*reqs[0])
        t1 = s.submit(*reqs[1])
        with pytest.raises(qap.QapError) as e:
            s.submit(*reqs[2])
        assert e.value.code == qap.QAP_E_BUSY
        done = {}
        drive(s, [t0, t1], done)
        t2 = s.submit(*reqs[2])          # room again once the queue drained
        drive(s, [t2], done)
        assert done[t2][1] == alone(reqs[2])[1]


def test_cancel_queued_and_running():
    note("serve: cancel")
    reqs = make_reqs(12, [60, 70, 80, 90, 100], 3000, 4000)
    with qap.Server(1 << 27, 2, 0.05) as s:    # two slots: three requests wait in the queue
        tickets = [s.submit(*r) for r in reqs]
        s.step()                                 # the first two are now running
        assert s.cancel(tickets[1]) is True      # running
        assert s.cancel(tickets[3]) is True      # queued
        with pytest.raises(qap.QapError):
            s.cancel(tickets[3])                 # forgotten
        keep = [tickets[i] for i in (0, 2, 4)]
        done = {}
        drive(s, keep, done)
        st = s.stats()
        assert st["cancelled"] == 2 and st["running"] == 0 and st["queued"] == 0 and st["pool_used"] == 0
    for t, i in zip(keep, (0, 2, 4)):
        bp, bc, bd = alone(reqs[i])
        assert (done[t][0] == bp).all() and done[t][1] == bc and done[t][2] == bd


def test_one_failed_search_leaves_the_rest_serving():
    note("serve: injected failure")
    reqs = make_reqs(13, [30, 64, 100, 150, 200, 77], 2000, 4000)
    with qap.Server(1 << 28, 8, 0.05) as s:
        tickets = [s.submit(*r) for r in reqs]
        s.step()
        s.inject_failure(tickets[2])
        done, failed = {}, {}
        for _ in range(200000):
            s.step()
            for t in tickets:
                if t in done or t in failed:
                    continue
                try:
                    r = s.result(t)
                except qap.QapError as e:
                    failed[t] = e.code
                    continue
                if r is not None:
                    done[t] = r
            if len(done) + len(failed) == len(tickets):
                break
        assert failed == {tickets[2]: qap.QAP_E_DEVICE}
        st = s.stats()
        assert st["failed"] == 1 and st["finished"] == len(reqs) - 1 and st["pool_used"] == 0
    for i, t in enumerate(tickets):
        if i == 2:
            continue
        bp, bc, bd = alone(reqs[i])
        assert (done[t][0] == bp).all() and done[t][1] == bc and done[t][2] == bd


def test_admission_passes_over_a_request_that_does_not_fit():
    note("serve: admission past the head")
    big = make_reqs(14, [200, 210], 3000, 3000)
    small = make_reqs(15, [24, 26, 28], 100, 200)
    with qap.Server(1 << 30, 8, 0.05) as s:
        fb = s.footprint(200)
        fs = s.footprint(28)
    pool = fb + fb // 4 + 4 * fs     # room for one big request and the small ones, not two big ones
    with qap.Server(pool, 8, 0.05) as s:
        tb = [s.submit(*r) for r in big]
        ts = [s.submit(*r) for r in small]
        order, done = [], {}
        for _ in range(200000):
            s.step()
            for t in tb + ts:
                if t not in done:
                    r = s.result(t)
                    if r is not None:
                        done[t] = r
                        order.append(t)
            if len(done) == 5:
                break
        # the small requests, queued behind the second big one, finish before it
        assert order.index(tb[1]) > max(order.index(t) for t in ts)
    for t, r in zip(tb + ts, big + small):
        bp, bc, bd = alone(r)
        assert (done[t][0] == bp).all() and done[t][1] == bc and done[t][2] == bd


def test_background_thread_serves_a_mix():
    note("serve: background thread")
    reqs = make_reqs(16, [33, 48, 75, 120, 170, 230, 250, 61], 500, 3000)
    hs = [qap.Handle(F, D) for F, D, *_ in reqs[:4]]
    try:
        with qap.Server(1 << 28, 6, 0.2) as s:
            s.start()
            tickets = [s.submit_handle(h, r[2], *r[3:]) for h, r in zip(hs, reqs[:4])]
            for r in reqs[4:]:
                tickets.append(s.submit(*r))
                time.sleep(0.002)                # arrivals while chunks run
            got, t0 = {}, time.time()
            while len(got) < len(tickets):
                for t in tickets:
                    if t not in got:
                        r = s.poll(t)
                        if r is not None:
                            got[t] = r
                time.sleep(0.001)
                assert time.time() - t0 < 60, "the server thread made no progress"
            with pytest.raises(qap.QapError):
                s.step()                         # the thread steps it
            s.stop()
            assert s.stats()["finished"] == len(reqs)
        for t, r in zip(tickets, reqs):
            bp, bc, _ = alone(r)
            assert (got[t][0] == bp).all() and got[t][1] == bc
    finally:
        for h in hs:
            h.close()


def test_tabu_batch_per_instance_arrays():
    note("batch: per-instance arrays")
    rng = np.random.default_rng(17)
    sizes = [20, 45, 77, 130, 33]
    insts = [W.random_instance(rng, n, 0, 99) for n in sizes]
    ks = [3, 1, 2, 4, 2]
    perms = [W.starts(rng, n, k) for n, k in zip(sizes, ks)]
    lohi = [W.tabu_tenure_range(n) for n in sizes]
    seeds = [int(x) for x in rng.integers(0, 2**62, len(sizes))]
    hs = [qap.Handle(F, D) for F, D in insts]
    try:
        ps, bs = qap.tabu_batch_lists(hs, perms, 400, [a for a, _ in lohi], [b for _, b in lohi], seeds)
        cp, cb, _ = qap.tabu_batch(hs, np.concatenate([p.reshape(-1) for p in perms]), ks, 400,
                                   [a for a, _ in lohi], [b for _, b in lohi], seeds)
        assert (np.concatenate([p.reshape(-1) for p in ps]) == cp).all()
        assert (np.concatenate(bs) == cb).all()
        F, D = insts[3]
        for j in range(ks[3]):
            obp, obc, _, _ = oracle.tabu(F, D, perms[3][j], 400, lohi[3][0], lohi[3][1], seeds[3], j)
            assert (ps[3][j] == obp).all() and bs[3][j] == obc
    finally:
        for h in hs:
            h.close()


def test_served_frequency_memory_equals_the_oracle():
    """Requests that keep the frequency memory (qap_server_submit_freq), with and without
    the diversification move and with each tabu attribute, served in small chunks beside
    plain requests: every result and every count equals oracle.tabu_freq (plain ones
    oracle.tabu), so the counts, unit marks, unit-location table and the iteration of the
    last new best survive the chunk boundaries."""
    rng = np.random.default_rng(771)
    # (n, iters, div, attr, symmetric); the streamed form at n = 200
    spec = [(40, 900, 0, 0, False), (64, 700, 25, 0, True), (97, 600, 30, 1, False), (33, 800, 0, 2, False),
            (150, 400, 20, 2, False), (200, 250, 15, 1, True), (71, 500, 0, 1, False)]
    reqs = []
    for n, it, div, attr, sym in spec:
        F, D = W.random_instance(rng, n, 0, 99, symmetric=sym)
        lo, hi = (3, 3 + n // 10) if attr == 1 else W.paper_tenure_range(n)
        reqs.append((F, D, W.starts(rng, n, 1)[0], it, lo, hi, int(rng.integers(0, 2**62)), div, attr))
    plain = make_reqs(772, [50, 120], 300, 600)
    note("served frequency memory: %d requests" % (len(reqs) + len(plain)))
    hs = [qap.Handle(q[0], q[1]) for q in reqs]
    out, outp = {}, {}
    with qap.Server(1 << 28, 16, 0.2) as s:
        tickets = [s.submit_freq(h, q[2], q[3], q[4], q[5], q[6], div=q[7], attr=q[8]) for h, q in zip(hs, reqs)]
        ptick = [s.submit(*q) for q in plain]
        with pytest.raises(qap.QapError) as ei:   # a plain request has no counts to give
            while s.poll_freq(ptick[0]) is None:
                s.step()
        assert ei.value.code == qap.QAP_E_INVALID
        for _ in range(200000):
            if len(out) == len(tickets) and len(outp) == len(ptick):
                break
            s.step()
            for t in tickets:
                if t not in out:
                    r = s.poll_freq(t)
                    if r is not None:
                        out[t] = r
            for t in ptick:
                if t not in outp:
                    r = s.poll(t)
                    if r is not None:
                        outp[t] = r
        assert s.stats()["steps"] > 3   # chunked
    for t, q in zip(tickets, reqs):
        F, D, p0, it, lo, hi, seed, div, attr = q
        bp, bc, _, freq, _ = oracle.tabu_freq(F, D, p0, it, lo, hi, seed, start=0, div=div, attr=attr)
        gp, gc, gf = out[t]
        assert (gp == bp).all() and gc == bc, (q[3], div, attr)
        assert (gf == freq).all(), (q[3], div, attr)
    for t, q in zip(ptick, plain):
        F, D, p0, it, lo, hi, seed = q
        bp, bc, _, _ = oracle.tabu(F, D, p0, it, lo, hi, seed, 0)
        assert (outp[t][0] == bp).all() and outp[t][1] == bc
    for h in hs:
        h.close()
