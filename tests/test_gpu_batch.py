"""GPU parity of the batched tabu search over many instances of uneven n.

The batched launch must give every start exactly what the oracle gives it alone (best
permutation, best cost, moves made), and exactly what a search of that instance alone on
the GPU gives (batch invariance).  The full-size uneven batch (512 instances, n from 20
to 150, 8 starts of 5000 iterations) is run as the benchmark runs it, inside a captured
HIP graph replayed several times, and a sample of its starts is recomputed by the oracle.
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


def oracle_rows(insts, ks, iters, lohi, seeds):
    """Every (instance, start) of a batch through the oracle, in batch order."""
    jobs = [(i, j) for i in range(len(insts)) for j in range(ks[i])]

    def one(a):
        i, j = a
        F, D, P = insts[i]
        return oracle.tabu(F, D, P[j], iters, lohi[i][0], lohi[i][1], seeds[i], j)

    return jobs, pmap(one, jobs)


def mixed_batch(seed, sizes, k):
    rng = np.random.default_rng(seed)
    insts, lohi, seeds = [], [], []
    for t, n in enumerate(sizes):
        F, D = W.random_instance(rng, n, 0, 99, symmetric=(t % 3 == 1), diag=(t % 4 == 2))
        insts.append((F, D, W.starts(rng, n, k[t])))
        lo, hi = W.tabu_tenure_range(n)
        lohi.append((lo, hi))
        seeds.append(int(rng.integers(0, 2**62)))
    return insts, lohi, seeds


@pytest.mark.parametrize("sizes,k,iters", [
    ([2, 3, 5, 12, 40, 64, 33, 150, 97, 128], [3, 2, 4, 1, 3, 2, 0, 2, 3, 2], 400),
    ([150, 149, 20, 21, 65, 66, 130], [2, 1, 3, 2, 2, 1, 2], 1500),
])
def test_batch_equals_oracle_mixed_n(sizes, k, iters):
    insts, lohi, seeds = mixed_batch(sum(sizes), sizes, k)
    note("batch mixed sizes=%s k=%s iters=%d" % (sizes, k, iters))
    hs = [qap.Handle(F, D) for F, D, _ in insts]
    perms = np.concatenate([P.reshape(-1) for _, _, P in insts]).astype(np.int32)
    p, c, d = qap.tabu_batch(hs, perms, k, iters, [a for a, _ in lohi], [b for _, b in lohi], seeds)
    jobs, res = oracle_rows(insts, k, iters, lohi, seeds)
    off = 0
    for (i, j), r in zip(jobs, res):
        n = insts[i][0].shape[0]
        row = sum(k[:i]) + j
        got = p[off:off + n]
        assert (got == r[0]).all() and c[row] == r[1] and d[row] == r[2], (i, j, n)
        off += n
    for h in hs:
        h.close()


def test_batch_every_kernel_variant_equals_oracle():
    """Shapes chosen so that every batched kernel variant runs: tiles of 2 rows on 128,
    256 and 512 lanes, of 4 rows on 256, 512 and 768, of 8 rows, and the streamed form (a
    search gets the smallest workgroup with a lane per tile and per (index, family) task)."""
    sizes = [30, 60, 50, 100, 70, 130, 190, 140]
    rows = [2, 2, 4, 4, 2, 8, -8, 4]
    lanes = [128, 256, 256, 512, 512, 512, 512, 768]
    k = [2, 2, 2, 2, 2, 1, 1, 2]
    iters = 300
    insts, lohi, seeds = mixed_batch(7 + sum(sizes), sizes, k)
    note("batch variants sizes=%s rows=%s" % (sizes, rows))
    hs = [qap.Handle(F, D) for F, D, _ in insts]
    for h, r, want in zip(hs, rows, lanes):
        h.set_tile_rows("batch", r)
        assert h.tile_rows("batch") == (r, want), (h.n, r)
    perms = np.concatenate([P.reshape(-1) for _, _, P in insts]).astype(np.int32)
    p, c, d = qap.tabu_batch(hs, perms, k, iters, [a for a, _ in lohi], [b for _, b in lohi], seeds)
    jobs, res = oracle_rows(insts, k, iters, lohi, seeds)
    off = 0
    for (i, j), r in zip(jobs, res):
        n = insts[i][0].shape[0]
        row = sum(k[:i]) + j
        assert (p[off:off + n] == r[0]).all() and c[row] == r[1] and d[row] == r[2], (i, j, n)
        off += n
    for h in hs:
        h.close()


@pytest.mark.parametrize("lanes", [1, 2, 3, 5])
def test_batch_side_stream_plan_does_not_change_results(lanes, monkeypatch):
    """The batched launch deals its kernel variants to side streams (QAP_BATCH_LANES
    overrides how many, read when the plan is made); one lane runs them all back to back,
    five is more lanes than there are variants here.  Every count gives the oracle's
    results, eagerly and from a captured graph replayed twice."""
    import torch
    monkeypatch.setenv("QAP_BATCH_LANES", str(lanes))
    sizes = [30, 60, 50, 100, 130, 140]
    rows = [2, 2, 4, 4, 4, 4]
    k = [2, 2, 2, 2, 1, 2]
    iters = 200
    insts, lohi, seeds = mixed_batch(31 + sum(sizes), sizes, k)
    note("batch side-stream lanes=%d sizes=%s" % (lanes, sizes))
    hs = [qap.Handle(F, D) for F, D, _ in insts]
    for h, r in zip(hs, rows):
        h.set_tile_rows("batch", r)
    starts = torch.from_numpy(np.concatenate([P.reshape(-1) for _, _, P in insts]).astype(np.int32)).cuda()
    jobs, res = oracle_rows(insts, k, iters, lohi, seeds)
    with qap.Batch(hs, k, iters, [a for a, _ in lohi], [b for _, b in lohi], seeds) as b:
        want = {variant_of(n, r, t % 3 == 1) for t, (n, r) in enumerate(zip(sizes, rows))}
        assert b.groups() == len(want) == 5, want   # r2 on 128/256 lanes, r4 on 256/512/768
        stream = torch.cuda.Stream()
        work = torch.empty_like(starts)
        best = torch.empty(sum(k), dtype=torch.int64, device="cuda")
        done = torch.empty(sum(k), dtype=torch.int32, device="cuda")
        outs = []
        with torch.cuda.stream(stream):
            work.copy_(starts)
            b.run_async(work, best, done, stream=stream)
        torch.cuda.synchronize()
        outs.append((work.cpu().numpy(), best.cpu().numpy(), done.cpu().numpy()))
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            work.copy_(starts)
            b.run_async(work, best, done, stream=stream)
        for _ in range(2):
            work.fill_(0)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            outs.append((work.cpu().numpy(), best.cpu().numpy(), done.cpu().numpy()))
    for p, c, d in outs:
        off = 0
        for (i, j), r in zip(jobs, res):
            n = insts[i][0].shape[0]
            row = sum(k[:i]) + j
            assert (p[off:off + n] == r[0]).all() and c[row] == r[1] and d[row] == r[2], (lanes, i, j, n)
            off += n
    for h in hs:
        h.close()


def test_batch_invariance_against_single_instance_searches():
    w = W.c4_batch(m=24, k=4, iters=1200)
    note("batch invariance: 24 instances of the uneven workload, 4 starts x 1200 iterations")
    hs = [qap.Handle(I.F, I.D) for I in w.instances]
    lo = [w.tenure(I.n)[0] for I in w.instances]
    hi = [w.tenure(I.n)[1] for I in w.instances]
    seeds = [I.seed for I in w.instances]
    perms = np.concatenate([I.perms.reshape(-1) for I in w.instances])
    p, c, d = qap.tabu_batch(hs, perms, [4] * 24, w.iters, lo, hi, seeds)
    off, row = 0, 0
    for t, I in enumerate(w.instances):
        sp, sc, sd = hs[t].tabu(I.perms, w.iters, lo[t], hi[t], I.seed)
        n = I.n
        assert (p[off:off + 4 * n].reshape(4, n) == sp).all(), t
        assert (c[row:row + 4] == sc).all() and (d[row:row + 4] == sd).all(), t
        off += 4 * n
        row += 4
    for h in hs:
        h.close()


def test_batch_rejects_unsupported_and_bad_input():
    rng = np.random.default_rng(5)
    F, D = W.random_instance(rng, 256, 0, 99)
    with qap.Handle(F, D) as big, qap.Handle(*W.random_instance(rng, 10, 0, 9)) as small:
        with pytest.raises(qap.QapError) as ei:   # register tiles of 2 rows cannot hold n = 256
            qap.Batch([small, big], [1, 1], 100, [1, 1], [3, 30], [1, 2], rows=[2, 2])
        assert ei.value.code == qap.QAP_E_UNSUPPORTED
        with pytest.raises(qap.QapError) as ei:   # 16-row tiles do not exist in the batched kernel
            qap.Batch([small], [1], 100, [1], [3], [1], rows=[16])
        assert ei.value.code == qap.QAP_E_UNSUPPORTED
        bad = np.arange(10, dtype=np.int32)
        bad[3] = 4
        with pytest.raises(qap.QapError) as ei:
            qap.tabu_batch([small], bad, [1], 100, [1], [3], [1])
        assert ei.value.code == qap.QAP_E_NOT_PERM
        with qap.Batch([small], [0], 100, [1], [3], [1]) as b:   # empty batch runs as a no-op
            assert b.starts == 0 and b.perm_ints == 0


def test_batch_full_size_graph_replay_sampled():
    import torch
    w = W.c4_batch()
    insts = w.instances
    m, k = len(insts), len(insts[0].perms)
    note("batch full size: %d instances x %d starts x %d iterations, graph replay" % (m, k, w.iters))
    hs = [qap.Handle(I.F, I.D) for I in insts]
    lo = [w.tenure(I.n)[0] for I in insts]
    hi = [w.tenure(I.n)[1] for I in insts]
    seeds = [I.seed for I in insts]
    starts = torch.from_numpy(np.concatenate([I.perms.reshape(-1) for I in insts])).cuda()
    work = torch.empty_like(starts)
    best = torch.empty(m * k, dtype=torch.int64, device="cuda")
    done = torch.empty(m * k, dtype=torch.int32, device="cuda")
    with qap.Batch(hs, [k] * m, w.iters, lo, hi, seeds) as b:
        assert b.starts == m * k and b.perm_ints == starts.numel()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            work.copy_(starts)
            b.run_async(work, best, done, stream=s)
        torch.cuda.synchronize()
        ep, ec, ed = work.cpu().numpy(), best.cpu().numpy(), done.cpu().numpy()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            work.copy_(starts)
            b.run_async(work, best, done, stream=s)
        for rep in range(3):
            best.fill_(-1)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert (work.cpu().numpy() == ep).all() and (best.cpu().numpy() == ec).all(), rep
            assert (done.cpu().numpy() == ed).all(), rep
    assert (ed <= w.iters).all() and (ed >= 0).all()
    off = np.concatenate([[0], np.cumsum([k * I.n for I in insts])])
    for t, I in enumerate(insts):
        rows = ep[off[t]:off[t + 1]].reshape(k, I.n)
        assert (hs[t].cost(rows) == ec[t * k:(t + 1) * k]).all(), t
    sample = [(0, 0), (1, 7), (2, 3), (257, 5), (510, 1), (511, 6)]
    sample += [(int(np.argmax([I.n for I in insts])), 2)]

    def one(a):
        t, j = a
        I = insts[t]
        return oracle.tabu(I.F, I.D, I.perms[j], w.iters, lo[t], hi[t], I.seed, j)

    for (t, j), r in zip(sample, pmap(one, sample)):
        n = insts[t].n
        got = ep[off[t] + j * n: off[t] + (j + 1) * n]
        assert (got == r[0]).all() and ec[t * k + j] == r[1] and ed[t * k + j] == r[2], (t, j)
    for h in hs:
        h.close()


# Variant order of qap_batch_groups: tiles of 2, 4, 8 rows on 512 lanes, streamed, 2 rows on
# 128 and 256 lanes, 4 rows on 256 and 768 lanes.
VARIANTS = ["r2", "r4", "r8", "stream", "r2_128", "r2_256", "r4_256", "r4_768"]


def tile_count(n, rows):
    """Register tiles of rows x 4 that hold some move u < v."""
    return sum(1 for g in range((n + rows - 1) // rows) for b in range((n + 3) // 4)
               if g * rows < min(4 * b + 4, n) - 1)


def variant_of(n, rows, sym):
    """The batched kernel a search of this n and tile shape runs on (a lane per tile and per
    (index, family) task, the smallest workgroup that holds them)."""
    if rows < 0:
        return "stream"
    nt = tile_count(n, rows)
    need = max(nt, (2 if sym else 4) * n)
    if rows == 2:
        return "r2_128" if need <= 128 else ("r2_256" if need <= 256 else "r2")
    if rows == 4:
        return "r4_256" if need <= 256 else ("r4" if need <= 512 else "r4_768")
    return "r8"


def test_batch_full_size_every_variant_sampled():
    """The full uneven batch with tile shapes spread over every batched kernel variant
    (rows forced per instance in rotation, the first that fits), run once; 8 (instance,
    start) pairs of every variant are recomputed by the oracle."""
    import torch
    w = W.c4_batch()
    insts = w.instances
    m, k = len(insts), len(insts[0].perms)
    note("batch full size, every variant: %d instances x %d starts x %d iterations" % (m, k, w.iters))
    hs = [qap.Handle(I.F, I.D) for I in insts]
    order = [[2, 4, 8, -8], [4, 8, -8], [8, -8], [-8]]
    rows, kind = [], []
    for t, (I, h) in enumerate(zip(insts, hs)):
        for r in order[t % 4]:
            try:
                h.set_tile_rows("batch", r)
            except qap.QapError:
                continue
            rows.append(r)
            break
        sym = bool((I.F == I.F.T).all() and (I.D == I.D.T).all())
        kind.append(variant_of(I.n, rows[-1], sym))
    lo = [w.tenure(I.n)[0] for I in insts]
    hi = [w.tenure(I.n)[1] for I in insts]
    seeds = [I.seed for I in insts]
    work = torch.from_numpy(np.concatenate([I.perms.reshape(-1) for I in insts])).cuda()
    best = torch.empty(m * k, dtype=torch.int64, device="cuda")
    done = torch.empty(m * k, dtype=torch.int32, device="cuda")
    with qap.Batch(hs, [k] * m, w.iters, lo, hi, seeds) as b:
        _, counts = b.groups(counts=True)
        expect = [k * kind.count(v) for v in VARIANTS]
        assert list(counts[:len(VARIANTS)]) == expect, (list(counts), expect)
        assert all(c > 0 for c in counts[:len(VARIANTS)]), counts
        assert counts[len(VARIANTS)] == 0   # no instance above n = 256 here
        b.run_async(work, best, done)
        torch.cuda.synchronize()
    ep, ec, ed = work.cpu().numpy(), best.cpu().numpy(), done.cpu().numpy()
    off = np.concatenate([[0], np.cumsum([k * I.n for I in insts])])
    rng = np.random.default_rng(4)
    sample = []
    for v in VARIANTS:
        ts = [t for t in range(m) if kind[t] == v]
        pick = rng.choice(len(ts), size=min(8, len(ts)), replace=False)
        sample += [(ts[int(i)], int(rng.integers(0, k))) for i in pick]
    assert len(sample) >= 64

    def one(a):
        t, j = a
        I = insts[t]
        return oracle.tabu(I.F, I.D, I.perms[j], w.iters, lo[t], hi[t], I.seed, j)

    for (t, j), r in zip(sample, pmap(one, sample)):
        n = insts[t].n
        got = ep[off[t] + j * n: off[t] + (j + 1) * n]
        assert (got == r[0]).all() and ec[t * k + j] == r[1] and ed[t * k + j] == r[2], (t, j, kind[t])
    for h in hs:
        h.close()


@pytest.mark.parametrize("n,sym", [(24, False), (64, False), (100, True), (150, False)])
def test_tuner_picks_a_fitting_shape_and_results_do_not_change(n, sym):
    rng = np.random.default_rng(n)
    F, D = W.random_instance(rng, n, 0, 99, symmetric=sym)
    perms = W.starts(rng, n, 3)
    lo, hi = W.tabu_tenure_range(n)
    note("tuner n=%d sym=%s" % (n, sym))
    with qap.Handle(F, D) as h:
        ref = h.tabu(perms, 300, lo, hi, 11)
        for algo in ("tabu", "2opt", "batch"):
            rows, times = h.tune_tile_rows(algo, k=32, iters=100)
            assert rows in times and all(t > 0 for t in times.values()), (algo, times)
            assert rows == min(times, key=times.get)
            assert h.tile_rows(algo)[0] == rows
        got = h.tabu(perms, 300, lo, hi, 11)
        assert all((a == b).all() for a, b in zip(ref, got))
        p, c, d = qap.tabu_batch([h], perms.reshape(-1), [3], 300, [lo], [hi], [11])
        assert (p.reshape(3, n) == ref[0]).all() and (c == ref[1]).all() and (d == ref[2]).all()


def test_tile_cache_round_trip(tmp_path):
    from paper_2307_11248_amd.autotune import TileCache
    rng = np.random.default_rng(3)
    insts = [W.random_instance(rng, n, 0, 99) for n in (30, 30, 77)]
    hs = [qap.Handle(F, D) for F, D in insts]
    path = str(tmp_path / "tiles.json")
    note("tile cache round trip")
    c1 = TileCache(path, k=32, iters=100)
    rows1 = c1.apply_all(hs, "batch")
    c1.save()
    assert c1.tuned == 2 and rows1[0] == rows1[1]
    c2 = TileCache(path, k=32, iters=100)
    rows2 = c2.apply_all(hs, "batch")
    assert c2.tuned == 0 and rows2 == rows1
    assert [h.tile_rows("batch")[0] for h in hs] == rows1
    for h in hs:
        h.close()


@pytest.mark.parametrize("sizes,k,iters,divs,attrs", [
    # every attribute and diversification in one batch, n across the register shapes
    ([12, 40, 64, 33, 97, 128, 150, 5], [2, 2, 1, 2, 2, 1, 2, 3], 600,
     [0, 25, 0, 40, 30, 0, 50, 10], [0, 0, 1, 1, 2, 2, 0, 1]),
    # the streamed form (n above 176) beside register tiles, Zhu's short tenure for attr 1
    ([200, 180, 60, 21], [1, 2, 2, 2], 300, [0, 20, 15, 0], [2, 1, 0, 2]),
])
def test_batch_freq_equals_oracle(sizes, k, iters, divs, attrs):
    """Batched searches with the frequency memory, the diversification move and the unit
    attributes (qap_batch_create_freq) against oracle.tabu_freq start by start: best
    permutation, best cost, moves made and the exchange counts."""
    import torch
    insts, lohi, seeds = mixed_batch(7 * sum(sizes) + 1, sizes, k)
    for t, n in enumerate(sizes):
        if attrs[t] == 1 and t % 2 == 1:
            lohi[t] = (3, 3 + n // 10)
    note("batch freq sizes=%s k=%s iters=%d div=%s attr=%s" % (sizes, k, iters, divs, attrs))
    hs = [qap.Handle(F, D) for F, D, _ in insts]
    b = qap.Batch(hs, k, iters, [a for a, _ in lohi], [c for _, c in lohi], seeds, freq=True, div=divs, attr=attrs)
    perms = torch.from_numpy(np.concatenate([P.reshape(-1) for _, _, P in insts]).astype(np.int32)).cuda()
    best = torch.zeros(b.starts, dtype=torch.int64, device="cuda")
    done = torch.zeros(b.starts, dtype=torch.int32, device="cuda")
    freq = torch.full((b.freq_ints,), -1, dtype=torch.int32, device="cuda")
    b.run_async(perms, best, done)
    b.freq_async(freq)
    torch.cuda.synchronize()
    gp, gb, gd, gf = perms.cpu().numpy(), best.cpu().numpy(), done.cpu().numpy(), freq.cpu().numpy()
    jobs = [(i, j) for i in range(len(insts)) for j in range(k[i])]

    def one(a):
        i, j = a
        F, D, P = insts[i]
        return oracle.tabu_freq(F, D, P[j], iters, lohi[i][0], lohi[i][1], seeds[i], start=j, div=divs[i],
                                attr=attrs[i])

    res = pmap(one, jobs)
    po = fo = 0
    for t, ((i, j), r) in enumerate(zip(jobs, res)):
        n = sizes[i]
        m = n * (n - 1) // 2
        bp, bc, bd, bf, _ = r
        assert (gp[po:po + n] == bp).all(), "instance %d start %d: permutation" % (i, j)
        assert gb[t] == bc and gd[t] == bd, "instance %d start %d: (%d, %d) vs oracle (%d, %d)" % (
            i, j, gb[t], gd[t], bc, bd)
        assert (gf[fo:fo + m] == bf).all(), "instance %d start %d: exchange counts" % (i, j)
        po += n
        fo += m
    assert fo == b.freq_ints
    # a second run of the same plan resets the counts and gives the same results
    perms2 = torch.from_numpy(np.concatenate([P.reshape(-1) for _, _, P in insts]).astype(np.int32)).cuda()
    b.run_async(perms2, best, done)
    b.freq_async(freq)
    torch.cuda.synchronize()
    assert (perms2.cpu().numpy() == gp).all() and (freq.cpu().numpy() == gf).all()
    b.close()
    for h in hs:
        h.close()
