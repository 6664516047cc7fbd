"""GPU step records (qap_tabu_trace_async) against the oracle's, move by move.

The step record is the debugging aid for localising a divergence between the HIP path
and the oracle: the first step whose (r, s, delta, cost after) differs names the
iteration where the two searches part.  Every case here must have none; a second check
shows the helper finds the first differing step when two searches do part (different
tenure streams).
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


def first_divergence(a, b):
    """Index of the first step at which two step records differ (rows of (r, s, delta,
    cost after)), or None if the shorter one is a prefix of the other and they have
    the same length."""
    m = min(len(a), len(b))
    bad = np.nonzero((a[:m] != b[:m]).any(axis=1))[0]
    if len(bad):
        return int(bad[0])
    return None if len(a) == len(b) else m


def gpu_trace(F, D, perms, iters, lo, hi, seed, cap, div=0, attr=0, rows=None):
    import torch
    k, n = perms.shape
    with qap.Handle(F, D) as h:
        if rows is not None:
            h.set_tile_rows("tabu", rows)
        dp = torch.from_numpy(perms).cuda()
        db = torch.zeros(k, dtype=torch.int64, device="cuda")
        dd = torch.zeros(k, dtype=torch.int32, device="cuda")
        df = torch.zeros((k, n * (n - 1) // 2), dtype=torch.int32, device="cuda")
        dt = torch.full((k, cap, 4), -1, dtype=torch.int64, device="cuda")
        h.tabu_trace_async(dp, iters, lo, hi, seed, db, df, dt, dd, div=div, attr=attr)
        torch.cuda.synchronize()
        return dp.cpu().numpy(), db.cpu().numpy(), dd.cpu().numpy(), dt.cpu().numpy()


# (n, k, iters, symmetric, div, attr, tile rows or None)
CASES = [
    (24, 3, 300, False, 0, 0, None),
    (40, 2, 500, True, 30, 0, 2),
    (64, 2, 400, False, 0, 1, 4),
    (97, 2, 300, False, 25, 2, 8),
    (200, 1, 150, False, 0, 0, -8),
    (300, 1, 80, True, 0, 1, None),
]


@pytest.mark.parametrize("n,k,iters,sym,div,attr,rows", CASES)
def test_trace_equals_oracle_step_by_step(n, k, iters, sym, div, attr, rows):
    note("trace n=%d k=%d iters=%d sym=%d div=%d attr=%d rows=%s" % (n, k, iters, sym, div, attr, rows))
    rng = np.random.default_rng(31 * n + attr)
    F, D = W.random_instance(rng, n, 0, 99, symmetric=sym)
    perms = W.starts(rng, n, k)
    lo, hi = (3, 3 + n // 10) if attr == 1 else W.paper_tenure_range(n)
    seed = 1234 + n
    cap = iters
    gp, gb, gd, gt = gpu_trace(F, D, perms, iters, lo, hi, seed, cap, div, attr, rows)
    for j in range(k):
        bp, bc, done, _, tr = oracle.tabu_freq(F, D, perms[j], iters, lo, hi, seed, start=j, div=div,
                                               trace_cap=cap, attr=attr)
        assert gd[j] == done
        got = gt[j, :gd[j]]
        step = first_divergence(got, tr)
        assert step is None, "start %d: first divergence at step %d: gpu %s oracle %s" % (
            j, step, got[step].tolist() if step < len(got) else None, tr[step].tolist() if step < len(tr) else None)
        assert (gt[j, gd[j]:] == -1).all()
        assert (gp[j] == bp).all() and gb[j] == bc


def test_trace_localises_a_divergence():
    """Two searches that differ only in their tenure stream agree up to some step and part
    there: the helper names that step, and every earlier step matches."""
    n, iters = 30, 400
    rng = np.random.default_rng(77)
    F, D = W.random_instance(rng, n, 0, 99)
    perms = W.starts(rng, n, 1)
    lo, hi = 2, 12
    _, _, gd, gt = gpu_trace(F, D, perms, iters, lo, hi, 5, iters)
    _, _, _, _, other = oracle.tabu_freq(F, D, perms[0], iters, lo, hi, 6, start=0, trace_cap=iters)
    got = gt[0, :gd[0]]
    step = first_divergence(got, other)
    assert step is not None and step > 0
    assert (got[:step] == other[:step]).all()
    assert (got[step] != other[step]).any()
