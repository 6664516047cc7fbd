"""GPU check of the parameter sweep's launches (paper_2307_11248_amd.sweep): a point of
the sweep, the best cost of k tabu searches from seeded starts with the paper's tenure
range, equals the oracle's best over the same starts, seed and range."""
import sys

import numpy as np
import pytest

import oracle
from paper_2307_11248_amd import sweep
from paper_2307_11248_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.init()
    yield


@pytest.mark.parametrize("name,k,iters,seed", [("a-like", 5, 150, 7), ("b-like", 6, 120, 21)])
def test_sweep_point_equals_oracle(name, k, iters, seed):
    F, D = sweep.stand_ins()[name]
    sys.__stderr__.write("[gpu-case] sweep point %s k=%d iters=%d seed=%d\n" % (name, k, iters, seed))
    sys.__stderr__.flush()
    r = sweep.Runner(F, D)
    try:
        best, ms = r.run(k, iters, seed)
    finally:
        r.close()
    starts = W.starts(np.random.default_rng(seed), sweep.N, k)
    lo, hi = W.paper_tenure_range(sweep.N)
    want = min(oracle.tabu(F, D, p, iters, lo, hi, seed, start=j)[1] for j, p in enumerate(starts))
    assert best == want and ms > 0
