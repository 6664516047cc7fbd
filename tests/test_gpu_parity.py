"""GPU parity: the HIP path against the CPU oracle, bit for bit (integer results).

Every case compares the same seeded inputs: costs, neighbourhood tables, 2opt local
optima (permutation, cost, number of moves) and tabu results (best permutation, best
cost, moves made).  Full-size workloads are run in the launch configuration the
benchmark times, and a sample of their starts is recomputed by the oracle.
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


def rand_inst(seed, n, sym=False, diag=False, hi=99):
    rng = np.random.default_rng(seed)
    F, D = W.random_instance(rng, n, 0, hi, symmetric=sym, diag=diag)
    return F, D, rng


def oracle_2opt_many(F, D, perms, max_iters=0):
    res = pmap(lambda p: oracle.two_opt(F, D, p, max_iters=max_iters), list(perms))
    return (np.stack([r[0] for r in res]), np.array([r[1] for r in res]), np.array([r[2] for r in res]))


def oracle_tabu_many(F, D, perms, iters, lo, hi, seed, start_ids):
    res = pmap(lambda a: oracle.tabu(F, D, a[0], iters, lo, hi, seed, a[1]), list(zip(perms, start_ids)))
    return (np.stack([r[0] for r in res]), np.array([r[1] for r in res]), np.array([r[2] for r in res]))


SIZES = [(2, False, False), (3, False, True), (4, True, False), (5, False, False), (7, False, True),
         (12, True, False), (17, False, False), (31, False, True), (64, False, False), (100, True, False),
         (130, False, False), (150, False, True), (193, True, False), (256, True, False)]


@pytest.mark.parametrize("n,sym,diag", SIZES)
def test_cost_and_table_parity(n, sym, diag):
    note("cost/table n=%d sym=%s diag=%s" % (n, sym, diag))
    F, D, rng = rand_inst(1000 + n, n, sym, diag, hi=255)
    perms = W.starts(rng, n, 5)
    with qap.Handle(F, D) as h:
        costs = h.cost(perms)
        tab = h.delta_table(perms)
    for j in range(5):
        assert costs[j] == oracle.cost(F, D, perms[j])
        assert (tab[j].astype(np.int64) == oracle.delta_table(F, D, perms[j])).all()


def test_two_opt_config1_full():
    note("2opt c1 n=12 k=32")
    w = W.c1_grid12()
    I = w.instances[0]
    with qap.Handle(I.F, I.D) as h:
        p, c, st = h.two_opt(I.perms)
    ep, ec, est = oracle_2opt_many(I.F, I.D, I.perms)
    assert (p == ep).all() and (c == ec).all() and (st == est).all()


def tile_shapes(h, algo):
    """Every tile shape that serves this n: register tiles of 1, 2, 4, 8, 16 rows, and the
    streamed kernel (-8: tiles of 8 rows kept in global memory between passes)."""
    out = []
    for rows in (1, 2, 4, 8, 16, -8):
        try:
            h.set_tile_rows(algo, rows)
            out.append(rows)
        except qap.QapError:
            pass
    h.set_tile_rows(algo, 0)
    return out


def test_automatic_shape_per_launch():
    """Without a shape set, each launch picks its tile from its number of starts (fewest
    rounds of workgroups over the compute units, ties to the smallest tile): a launch of
    one start reports the handle's shape, an explicit shape holds for every launch size,
    and the 1024-start 2opt launch of the n = 128 workload returns what every explicit
    shape returns, and what the oracle returns on a sample."""
    w = W.c3_euclid128_2opt(k=1024)
    I = w.instances[0]
    note("automatic shape n=128 k=1024")
    with qap.Handle(I.F, I.D) as h:
        shapes = tile_shapes(h, "2opt")
        for algo in ("tabu", "2opt"):
            assert h.launch_tile_rows(algo, 1) == h.tile_rows(algo)
            for k in (1, 256, 1024, 4096):
                assert h.launch_tile_rows(algo, k)[0] in tile_shapes(h, algo)
        h.set_tile_rows("2opt", shapes[-1])
        assert all(h.launch_tile_rows("2opt", k)[0] == shapes[-1] for k in (1, 1024))
        h.set_tile_rows("2opt", 0)
        p, c, st = h.two_opt(I.perms)
        for rows in shapes:
            h.set_tile_rows("2opt", rows)
            pe, ce, ste = h.two_opt(I.perms[:64])
            assert (pe == p[:64]).all() and (ce == c[:64]).all() and (ste == st[:64]).all(), rows
        h.set_tile_rows("2opt", 0)
    ep, ec, est = oracle_2opt_many(I.F, I.D, I.perms[::256])
    assert (p[::256] == ep).all() and (c[::256] == ec).all() and (st[::256] == est).all()


@pytest.mark.parametrize("n,sym,diag", [(2, False, False), (3, False, False), (4, True, True), (5, False, False),
                                        (9, False, True), (13, True, False), (17, False, False),
                                        (40, False, True), (64, True, False), (101, False, False),
                                        (150, False, False)])
def test_two_opt_parity_every_tile_shape(n, sym, diag):
    F, D, rng = rand_inst(2000 + n, n, sym, diag)
    perms = W.starts(rng, n, 6)
    ep, ec, est = oracle_2opt_many(F, D, perms)
    with qap.Handle(F, D) as h:
        for rows in tile_shapes(h, "2opt"):
            note("2opt n=%d rows=%d" % (n, rows))
            h.set_tile_rows("2opt", rows)
            p, c, st = h.two_opt(perms)
            assert (c == ec).all() and (st == est).all() and (p == ep).all(), rows


def test_two_opt_move_cap():
    F, D, rng = rand_inst(77, 30)
    perms = W.starts(rng, 30, 4)
    ep, ec, est = oracle_2opt_many(F, D, perms, max_iters=5)
    note("2opt cap n=30")
    with qap.Handle(F, D) as h:
        p, c, st = h.two_opt(perms, max_iters=5)
    assert (p == ep).all() and (c == ec).all() and (st == est).all()


@pytest.mark.parametrize("n,sym,diag,lohi,iters", [
    (3, False, False, (0, 1), 40), (4, False, True, (1, 2), 60), (6, True, False, (2, 4), 200),
    (9, False, False, (3, 6), 300), (16, False, True, (2, 6), 400), (23, True, False, (20, 25), 400),
    (37, False, False, (33, 40), 500), (64, False, False, (57, 70), 600), (90, True, False, (9, 29), 300),
    (128, False, True, (115, 140), 300), (150, False, False, (135, 165), 250)])
def test_tabu_parity_every_tile_shape(n, sym, diag, lohi, iters):
    F, D, rng = rand_inst(3000 + n, n, sym, diag)
    perms = W.starts(rng, n, 4)
    lo, hi = lohi
    seed = 4242 + n
    ep, ec, ed = oracle_tabu_many(F, D, perms, iters, lo, hi, seed, range(4))
    with qap.Handle(F, D) as h:
        for rows in tile_shapes(h, "tabu"):
            note("tabu n=%d rows=%d iters=%d" % (n, rows, iters))
            h.set_tile_rows("tabu", rows)
            p, c, d = h.tabu(perms, iters, lo, hi, seed)
            assert (c == ec).all() and (d == ed).all() and (p == ep).all(), rows


def test_tabu_constant_cost_tie_break():
    """F = J - I: every delta is 0, so the trajectory is decided by the tie-break and the
    tabu expiry alone; the best permutation must stay the start."""
    n = 16
    F = (np.ones((n, n)) - np.eye(n)).astype(np.int32)
    D = W.grid_manhattan(n)
    rng = np.random.default_rng(5)
    perms = W.starts(rng, n, 3)
    for lo, hi in ((5, 5), (3, 9), (0, 0)):
        ep, ec, ed = oracle_tabu_many(F, D, perms, 300, lo, hi, 8, range(3))
        note("tabu constant cost lo=%d hi=%d" % (lo, hi))
        with qap.Handle(F, D) as h:
            p, c, d = h.tabu(perms, 300, lo, hi, 8)
        assert (p == ep).all() and (c == ec).all() and (d == ed).all()
        assert (p == perms).all()


def test_tabu_premature_stop():
    for n in (3, 4, 5):
        F, D, rng = rand_inst(50 + n, n)
        perms = W.starts(rng, n, 3)
        ep, ec, ed = oracle_tabu_many(F, D, perms, 50, 100, 100, 3, range(3))
        note("tabu premature stop n=%d" % n)
        with qap.Handle(F, D) as h:
            p, c, d = h.tabu(perms, 50, 100, 100, 3)
        assert (d == ed).all() and (d < 50).all()
        assert (p == ep).all() and (c == ec).all()


def test_tabu_plain_equals_batched_and_start_ids():
    import torch
    F, D, rng = rand_inst(91, 48)
    perms = W.starts(rng, 48, 6)
    with qap.Handle(F, D) as h:
        outs = []
        for plain in (False, True):
            note("tabu plain=%s n=48" % plain)
            dp = torch.from_numpy(perms).cuda()
            db = torch.zeros(6, dtype=torch.int64, device="cuda")
            dd = torch.zeros(6, dtype=torch.int32, device="cuda")
            h.tabu_async(dp, 400, 43, 52, 11, db, dd, start_base=100, plain=plain)
            torch.cuda.synchronize()
            outs.append((dp.cpu().numpy(), db.cpu().numpy(), dd.cpu().numpy()))
        for j in (0, 3, 5):
            note("tabu alone start=%d" % j)
            dp = torch.from_numpy(perms[j:j + 1].copy()).cuda()
            db = torch.zeros(1, dtype=torch.int64, device="cuda")
            h.tabu_async(dp, 400, 43, 52, 11, db, None, start_base=100 + j)
            torch.cuda.synchronize()
            assert (dp.cpu().numpy()[0] == outs[0][0][j]).all() and db.item() == outs[0][1][j]
    for a, b in zip(outs[0], outs[1]):
        assert (a == b).all()
    ep, ec, ed = oracle_tabu_many(F, D, perms, 400, 43, 52, 11, range(100, 106))
    assert (outs[0][0] == ep).all() and (outs[0][1] == ec).all() and (outs[0][2] == ed).all()


def test_device_rejects_non_permutation_rows():
    import torch
    F, D, rng = rand_inst(17, 20)
    perms = W.starts(rng, 20, 3)
    bad = perms.copy()
    bad[1, 0] = bad[1, 1]
    with qap.Handle(F, D) as h:
        with pytest.raises(qap.QapError) as ei:
            h.tabu(bad, 10, 1, 2, 0)
        assert ei.value.code == qap.QAP_E_NOT_PERM
        note("device non-permutation row")
        dp = torch.from_numpy(bad).cuda()
        db = torch.zeros(3, dtype=torch.int64, device="cuda")
        dd = torch.zeros(3, dtype=torch.int32, device="cuda")
        h.tabu_async(dp, 100, 2, 5, 1, db, dd)
        torch.cuda.synchronize()
        d = dd.cpu().numpy()
        b = db.cpu().numpy()
        assert d[1] == qap.QAP_E_NOT_PERM and b[1] == np.iinfo(np.int64).min
        assert (dp.cpu().numpy()[1] == bad[1]).all()
        ep, ec, ed = oracle_tabu_many(F, D, bad[[0, 2]], 100, 2, 5, 1, [0, 2])
        assert (b[[0, 2]] == ec).all() and (d[[0, 2]] == ed).all()


# ---- full-size workloads, sampled starts recomputed by the oracle

def test_two_opt_config3_full_size_sampled():
    w = W.c3_euclid128_2opt()
    I = w.instances[0]
    note("2opt c3 n=128 k=1024")
    with qap.Handle(I.F, I.D) as h:
        p, c, st = h.two_opt(I.perms)
    sample = list(range(0, 1024, 43))
    ep, ec, est = oracle_2opt_many(I.F, I.D, I.perms[sample])
    assert (p[sample] == ep).all() and (c[sample] == ec).all() and (st[sample] == est).all()
    # every start: the result is a local optimum whose cost is Eq. (1) of its permutation
    with qap.Handle(I.F, I.D) as h:
        assert (h.cost(p) == c).all()
        assert (h.delta_table(p[:64]) >= 0).all()


def test_tabu_config2_full_size_sampled():
    import torch
    w = W.c2_dense64()
    I = w.instances[0]
    lo, hi = W.tabu_tenure_range(64)
    note("tabu c2 n=64 k=128 iters=20000")
    with qap.Handle(I.F, I.D) as h:
        dp = torch.from_numpy(I.perms).cuda()
        db = torch.zeros(128, dtype=torch.int64, device="cuda")
        dd = torch.zeros(128, dtype=torch.int32, device="cuda")
        h.tabu_async(dp, w.iters, lo, hi, I.seed, db, dd)
        torch.cuda.synchronize()
        p, c, d = dp.cpu().numpy(), db.cpu().numpy(), dd.cpu().numpy()
        assert (h.cost(p) == c).all()
    sample = list(range(128))   # every start
    ep, ec, ed = oracle_tabu_many(I.F, I.D, I.perms[sample], w.iters, lo, hi, I.seed, sample)
    assert (p[sample] == ep).all() and (c[sample] == ec).all() and (d[sample] == ed).all()
    assert (d == w.iters).all()


def test_tabu_config3_full_size_sampled():
    import torch
    w = W.c3_euclid128_tabu()
    I = w.instances[0]
    lo, hi = W.tabu_tenure_range(128)
    note("tabu c3 n=128 k=256 iters=10000")
    with qap.Handle(I.F, I.D) as h:
        dp = torch.from_numpy(I.perms).cuda()
        db = torch.zeros(256, dtype=torch.int64, device="cuda")
        dd = torch.zeros(256, dtype=torch.int32, device="cuda")
        h.tabu_async(dp, w.iters, lo, hi, I.seed, db, dd)
        torch.cuda.synchronize()
        p, c, d = dp.cpu().numpy(), db.cpu().numpy(), dd.cpu().numpy()
        assert (h.cost(p) == c).all()
    sample = list(range(0, 256, 8))   # 32 of the 256 starts
    ep, ec, ed = oracle_tabu_many(I.F, I.D, I.perms[sample], w.iters, lo, hi, I.seed, sample)
    assert (p[sample] == ep).all() and (c[sample] == ec).all() and (d[sample] == ed).all()


@pytest.mark.parametrize("n,sym,rows", [(12, False, 0), (40, True, 1), (64, False, 2), (130, False, 4),
                                        (200, False, -8), (300, False, -8)])
def test_tabu_frequency_memory_counts_the_oracle_moves(n, sym, rows):
    """The frequency memory (Sec. 4.3, lower triangle of Tabuarr) counts, per pair of
    locations, the exchanges the search made: it must equal the count of the oracle's
    moves, and keeping it must not change the search."""
    import torch
    F, D, rng = rand_inst(5000 + n, n, sym)
    k, iters, seed = 3, 250, 777
    perms = W.starts(rng, n, k)
    lo, hi = W.tabu_tenure_range(n)
    m = n * (n - 1) // 2
    note("tabu frequency memory n=%d rows=%d" % (n, rows))
    with qap.Handle(F, D) as h:
        if rows:
            h.set_tile_rows("tabu", rows)
        dp = torch.from_numpy(perms).cuda()
        db = torch.zeros(k, dtype=torch.int64, device="cuda")
        dd = torch.zeros(k, dtype=torch.int32, device="cuda")
        df = torch.full((k, m), -1, dtype=torch.int32, device="cuda")
        h.tabu_freq_async(dp, iters, lo, hi, seed, db, df, dd)
        torch.cuda.synchronize()
        got_p, got_c, got_d, got_f = dp.cpu().numpy(), db.cpu().numpy(), dd.cpu().numpy(), df.cpu().numpy()
    for j in range(k):
        bp, bc, done, tr = oracle.tabu(F, D, perms[j], iters, lo, hi, seed, start=j, trace_cap=iters)
        want = np.zeros(m, dtype=np.int64)
        for r, s, _, _ in tr:
            a, b = min(r, s), max(r, s)
            want[a * n - a * (a + 1) // 2 + (b - a - 1)] += 1
        assert (got_f[j] == want).all() and got_f[j].sum() == done, j
        assert (got_p[j] == bp).all() and got_c[j] == bc and got_d[j] == done, j


@pytest.mark.parametrize("n,sym,rows,div", [(12, False, 0, 3), (40, True, 1, 6), (64, False, 2, 10),
                                            (64, False, 1, 4), (101, True, 4, 8), (130, False, 8, 12),
                                            (150, False, 16, 9), (200, False, -8, 7), (230, True, -8, 11),
                                            (300, False, -8, 7), (420, True, -8, 3)])
def test_tabu_frequency_diversification_equals_oracle(n, sym, rows, div):
    """With div > 0 the frequency memory drives a diversification move (the least
    exchanged non-tabu pair after more than div iterations without a new best): best
    permutations, costs, moves made and counts equal the oracle's, on every tile shape,
    the streamed kernel included; the rule changes the search for at least one start."""
    import torch
    F, D, rng = rand_inst(6000 + n + div, n, sym)
    k, iters, seed = 4, 300, 4242
    perms = W.starts(rng, n, k)
    lo, hi = W.tabu_tenure_range(n)
    m = n * (n - 1) // 2
    note("tabu diversification n=%d rows=%d div=%d" % (n, rows, div))
    with qap.Handle(F, D) as h:
        if rows:
            h.set_tile_rows("tabu", rows)
        dp = torch.from_numpy(perms).cuda()
        db = torch.zeros(k, dtype=torch.int64, device="cuda")
        dd = torch.zeros(k, dtype=torch.int32, device="cuda")
        df = torch.full((k, m), -1, dtype=torch.int32, device="cuda")
        h.tabu_freq_async(dp, iters, lo, hi, seed, db, df, dd, div=div)
        torch.cuda.synchronize()
        got_p, got_c, got_d, got_f = dp.cpu().numpy(), db.cpu().numpy(), dd.cpu().numpy(), df.cpu().numpy()
    changed = False
    for j in range(k):
        bp, bc, done, freq, _ = oracle.tabu_freq(F, D, perms[j], iters, lo, hi, seed, start=j, div=div)
        assert (got_p[j] == bp).all() and got_c[j] == bc and got_d[j] == done, j
        assert (got_f[j] == freq).all(), j
        plain = oracle.tabu_freq(F, D, perms[j], iters, lo, hi, seed, start=j, div=0)
        changed |= not (plain[3] == freq).all()
    assert changed


@pytest.mark.parametrize("n,sym,rows,div", [(12, False, 0, 0), (40, True, 1, 0), (64, False, 2, 6),
                                            (101, True, 4, 0), (130, False, 8, 9), (150, False, 16, 0),
                                            (200, False, -8, 0), (210, True, -8, 8), (333, False, -8, 6)])
def test_tabu_unit_marking_equals_oracle(n, sym, rows, div):
    """The unit-marking tabu attribute (the two units moved are marked for the tenure; a
    move is tabu while either of its units is marked), alone and with the diversification
    move, equals the oracle on every tile shape, the streamed kernel included; it changes
    the search for at least one start."""
    import torch
    F, D, rng = rand_inst(7000 + n + div, n, sym)
    k, iters, seed = 3, 250, 99
    perms = W.starts(rng, n, k)
    lo, hi = 3, 3 + n // 10          # the short unit tenure of Zhu et al.
    m = n * (n - 1) // 2
    note("tabu unit marking n=%d rows=%d div=%d" % (n, rows, div))
    with qap.Handle(F, D) as h:
        if rows:
            h.set_tile_rows("tabu", rows)
        dp = torch.from_numpy(perms).cuda()
        db = torch.zeros(k, dtype=torch.int64, device="cuda")
        dd = torch.zeros(k, dtype=torch.int32, device="cuda")
        df = torch.full((k, m), -1, dtype=torch.int32, device="cuda")
        h.tabu_freq_async(dp, iters, lo, hi, seed, db, df, dd, div=div, attr=1)
        torch.cuda.synchronize()
        got_p, got_c, got_d, got_f = dp.cpu().numpy(), db.cpu().numpy(), dd.cpu().numpy(), df.cpu().numpy()
    changed = False
    for j in range(k):
        bp, bc, done, freq, _ = oracle.tabu_freq(F, D, perms[j], iters, lo, hi, seed, start=j, div=div, attr=1)
        assert (got_p[j] == bp).all() and got_c[j] == bc and got_d[j] == done, j
        assert (got_f[j] == freq).all(), j
        pair = oracle.tabu_freq(F, D, perms[j], iters, lo, hi, seed, start=j, div=div)
        changed |= not (pair[3] == freq).all()
    assert changed


@pytest.mark.parametrize("n,sym,rows,div", [(12, False, 0, 0), (40, True, 1, 0), (64, False, 2, 7),
                                            (101, True, 4, 0), (130, False, 8, 10), (150, False, 16, 0),
                                            (200, False, -8, 0), (190, False, -8, 9), (300, False, -8, 3)])
def test_tabu_unit_location_equals_oracle(n, sym, rows, div):
    """The unit-location tabu attribute (a move is tabu when both units would return to a
    location they left within their tenure), alone and with the diversification move,
    equals the oracle on every tile shape, the streamed kernel included; it changes the
    search for at least one start."""
    import torch
    F, D, rng = rand_inst(8000 + n + div, n, sym)
    k, iters, seed = 3, 250, 123
    perms = W.starts(rng, n, k)
    lo, hi = W.tabu_tenure_range(n)
    m = n * (n - 1) // 2
    note("tabu unit-location n=%d rows=%d div=%d" % (n, rows, div))
    with qap.Handle(F, D) as h:
        if rows:
            h.set_tile_rows("tabu", rows)
        dp = torch.from_numpy(perms).cuda()
        db = torch.zeros(k, dtype=torch.int64, device="cuda")
        dd = torch.zeros(k, dtype=torch.int32, device="cuda")
        df = torch.full((k, m), -1, dtype=torch.int32, device="cuda")
        h.tabu_freq_async(dp, iters, lo, hi, seed, db, df, dd, div=div, attr=2)
        torch.cuda.synchronize()
        got_p, got_c, got_d, got_f = dp.cpu().numpy(), db.cpu().numpy(), dd.cpu().numpy(), df.cpu().numpy()
    changed = False
    for j in range(k):
        bp, bc, done, freq, _ = oracle.tabu_freq(F, D, perms[j], iters, lo, hi, seed, start=j, div=div, attr=2)
        assert (got_p[j] == bp).all() and got_c[j] == bc and got_d[j] == done, j
        assert (got_f[j] == freq).all(), j
        pair = oracle.tabu_freq(F, D, perms[j], iters, lo, hi, seed, start=j, div=div)
        changed |= not (pair[3] == freq).all()
    assert changed
