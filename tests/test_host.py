"""CPU-side checks of the host logic around the kernels: the contraction identity the
neighbourhood-table kernel evaluates (against the oracle's Eq. (2) tables), the seeded
workload generators, the tile-shape cache of the autotuner, and bench.py's refusal of
more than one GPU.  None of these needs a GPU."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2307_11248_amd import qap
from paper_2307_11248_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def contraction_table(F, D, p):
    """delta(i, j) = T_ij + T_ji - T_ii - T_jj + c_ij with G = F[p][p], T = G D^T + G^T D,
    c_ij the k = i, j terms (the form the table kernel evaluates on the matrix cores)."""
    n = len(p)
    G = F[np.ix_(p, p)].astype(np.int64)
    Dm = D.astype(np.int64)
    T = G @ Dm.T + G.T @ Dm
    out = []
    for i in range(n):
        for j in range(i + 1, n):
            Dij, Dji, Dii, Djj = Dm[i, j], Dm[j, i], Dm[i, i], Dm[j, j]
            Gij, Gji, Gii, Gjj = G[i, j], G[j, i], G[i, i], G[j, j]
            c = (-(Dji - Dii) * (Gii - Gji) - (Djj - Dij) * (Gij - Gjj) - (Dij - Dii) * (Gii - Gij)
                 - (Djj - Dji) * (Gji - Gjj) + (Dji - Dij) * (Gij - Gji) + (Djj - Dii) * (Gii - Gjj))
            out.append(T[i, j] + T[j, i] - T[i, i] - T[j, j] + c)
    return np.array(out, dtype=np.int64)


@pytest.mark.parametrize("n,sym,diag", [(2, False, True), (3, False, True), (7, True, True), (20, False, False),
                                        (33, False, True)])
def test_contraction_identity_matches_eq2(n, sym, diag):
    rng = np.random.default_rng(100 + n)
    F, D = W.random_instance(rng, n, 0, 255, symmetric=sym, diag=diag)
    for p in W.starts(rng, n, 3):
        assert (contraction_table(F, D, p) == oracle.delta_table(F, D, p)).all()


def test_contraction_offsets_are_exact_in_int32():
    """The kernel shifts u8 entries by -128 and undoes it with row sums; at the largest n
    and entries every intermediate stays inside int32."""
    n, m = 256, 255
    acc = 2 * 2 * n * 128 * 128           # two phases, two products per tile pair
    shift = 128 * 2 * (4 * n * 128)       # 128 * (U_i + U_j), |U| <= 4 n 128
    const = 4 * 16384 * n
    assert acc + shift + const < 2**31
    assert (2 * n - 2) * m * m < 2**26    # |delta| bound used by the packed slot keys


def test_workload_generators_are_seeded_and_shaped():
    a, b = W.c4_batch(m=40), W.c4_batch(m=40)
    assert len(a.instances) == 40 and a.iters == 5000
    for x, y in zip(a.instances, b.instances):
        assert x.n == y.n and (x.F == y.F).all() and (x.D == y.D).all() and (x.perms == y.perms).all()
        assert 20 <= x.n <= 150 and x.perms.shape == (8, x.n)
        assert all(sorted(r) == list(range(x.n)) for r in x.perms)
        assert (np.diag(x.F) == 0).all() and (np.diag(x.D) == 0).all()
    reqs = W.c5_stream(count=60)
    t = [r.arrival_s for r in reqs]
    assert all(t1 > t0 for t0, t1 in zip(t, t[1:]))
    assert all(30 <= r.inst.n <= 256 and 2000 <= r.iters <= 20000 for r in reqs)
    w = W.c2_dense64()
    assert w.instances[0].perms.shape == (128, 64) and W.tabu_tenure_range(64) == (57, 70)


class _FakeHandle:
    """Stands in for qap.Handle: n, sym and the two tile-shape calls the cache uses."""

    def __init__(self, n, sym, fits=(2, 4, 8)):
        self.n, self.sym, self.fits = n, sym, fits
        self.rows, self.tuned = None, 0

    def set_tile_rows(self, algo, rows):
        if rows not in self.fits:
            raise qap.QapError.__new__(qap.QapError)
        self.rows = rows

    def tune_tile_rows(self, algo, k, iters):
        self.tuned += 1
        times = {r: 1.0 + abs(r - 4) for r in self.fits}
        self.rows = min(times, key=times.get)
        return self.rows, times


def test_tile_cache_keys_reuse_and_stale_entries(tmp_path, monkeypatch):
    from paper_2307_11248_amd import autotune
    monkeypatch.setattr(autotune, "_arch", lambda: "gfx950")
    monkeypatch.setattr(autotune, "_lib_digest", lambda: "lib1")
    path = str(tmp_path / "tiles.json")
    hs = [_FakeHandle(30, False), _FakeHandle(30, False), _FakeHandle(30, True), _FakeHandle(77, False)]
    c = autotune.TileCache(path)
    assert c.apply_all(hs, "batch") == [4, 4, 4, 4]
    assert c.tuned == 3 and hs[1].tuned == 0 and hs[1].rows == 4   # one measurement per (n, symmetric)
    c.save()
    c2 = autotune.TileCache(path)
    h = _FakeHandle(30, False)
    assert c2.apply(h, "batch") == 4 and h.tuned == 0 and c2.tuned == 0
    # a cached shape that no longer fits is measured again
    h2 = _FakeHandle(77, False, fits=(8,))
    assert c2.apply(h2, "batch") == 8 and h2.tuned == 1
    # another build of the library does not reuse the entries
    monkeypatch.setattr(autotune, "_lib_digest", lambda: "lib2")
    c3 = autotune.TileCache(path)
    h3 = _FakeHandle(30, False)
    c3.apply(h3, "batch")
    assert h3.tuned == 1


def test_sweep_quality_and_stand_ins():
    """The parameter sweep's host side: the quality gap, the best-of-k-seeds average, and
    the two n = 40 stand-in instances (uniform; sparse symmetric flows with Euclidean
    distances) with the paper's tenure range."""
    from paper_2307_11248_amd import sweep
    assert sweep.gap(110, 100) == 10.0 and sweep.gap(100, 100) == 0.0
    costs = [[120, 110, 130, 100], [105, 125, 100, 100]]
    assert sweep.seed_quality([c[:1] for c in costs], 100) == 12.5
    assert sweep.seed_quality([c[:2] for c in costs], 100) == 7.5
    assert sweep.seed_quality(costs, 100) == 0.0
    inst = sweep.stand_ins()
    (Fa, Da), (Fb, Db) = inst["a-like"], inst["b-like"]
    assert Fa.shape == Da.shape == (40, 40) and not (Fa == Fa.T).all()
    assert (Fb == Fb.T).all() and (Db == Db.T).all() and (Fb == 0).mean() > 0.5
    assert max(Fa.max(), Da.max(), Fb.max(), Db.max()) <= 255
    assert W.paper_tenure_range(40) == (4, 13)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
