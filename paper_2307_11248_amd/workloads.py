"""Seeded synthetic QAP instances and start permutations.

This module only draws inputs; it holds none of the method's arithmetic, and it is
the one piece of code that both the HIP path's callers and the CPU oracle's callers
use.  The instances stand in for the QAPLIB sets the paper measures on (Sec. 6.1.2):
uniform dense instances (like tai*a), sparse-flow instances with structured
distances (like tai*b), Manhattan grids and Euclidean point sets.

Every generator is ``numpy.random.Generator(Philox(key=SEED_BASE + config_id))``
and draws in a fixed order, so a configuration is reproducible from its id alone.
Distance and flow diagonals are zero in every configuration.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 230711248


def rng_for(config_id: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=SEED_BASE + int(config_id)))


def grid_manhattan(n: int) -> np.ndarray:
    """Manhattan distances of n locations laid row-major on a grid of width ceil(sqrt(n))."""
    w = int(math.ceil(math.sqrt(n)))
    i = np.arange(n)
    y, x = i // w, i % w
    return (np.abs(y[:, None] - y[None, :]) + np.abs(x[:, None] - x[None, :])).astype(np.int32)


def uniform_matrix(rng, n, lo, hi) -> np.ndarray:
    """Entries uniform in [lo, hi], zero diagonal, asymmetric."""
    m = rng.integers(lo, hi + 1, size=(n, n)).astype(np.int32)
    np.fill_diagonal(m, 0)
    return m


def sparse_matrix(rng, n, zero_frac, lo=1, hi=99) -> np.ndarray:
    """Each off-diagonal entry is 0 with probability zero_frac, else uniform in [lo, hi]."""
    vals = rng.integers(lo, hi + 1, size=(n, n)).astype(np.int32)
    keep = rng.random((n, n)) >= zero_frac
    m = np.where(keep, vals, 0).astype(np.int32)
    np.fill_diagonal(m, 0)
    return m


def symmetrise_upper(m: np.ndarray) -> np.ndarray:
    """Keep the strict upper triangle and mirror it (entries stay in their range)."""
    u = np.triu(m, 1)
    return (u + u.T).astype(np.int32)


def euclid_points(rng, n, side=100.0) -> np.ndarray:
    """Distances of n points uniform in a side x side square, rounded half away from zero."""
    pts = rng.uniform(0.0, side, size=(n, 2))
    h = np.hypot(pts[:, None, 0] - pts[None, :, 0], pts[:, None, 1] - pts[None, :, 1])
    return np.floor(h + 0.5).astype(np.int32)


def starts(rng, n, k) -> np.ndarray:
    """k start permutations, int32[k][n], each rng.permutation(n) in start order."""
    return np.stack([rng.permutation(n) for _ in range(k)]).astype(np.int32) if k else \
        np.zeros((0, n), dtype=np.int32)


def tabu_tenure_range(n: int) -> tuple[int, int]:
    """Tenure range [floor(0.9 n), floor(1.1 n)] used by every tabu workload here."""
    return (9 * n) // 10, (11 * n) // 10


def paper_tenure_range(n: int) -> tuple[int, int]:
    """The paper's own range [0.1 n, 0.33 n] (Sec. 4.3), floored."""
    return n // 10, (33 * n) // 100


@dataclass
class Instance:
    F: np.ndarray
    D: np.ndarray
    perms: np.ndarray
    seed: int = 0
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.F.shape[0])


@dataclass
class Workload:
    name: str
    algo: str                     # "2opt" or "tabu"
    instances: list = field(default_factory=list)
    iters: int = 0                # tabu iterations, or 2opt cap (0 = to local optimum)

    def tenure(self, n: int) -> tuple[int, int]:
        return tabu_tenure_range(n)


def c1_grid12(k: int = 32) -> Workload:
    """n=12 symmetric: F uniform [0,9] mirrored, D Manhattan on a 3x4 grid; 2opt from k starts."""
    rng = rng_for(1)
    n = 12
    F = symmetrise_upper(rng.integers(0, 10, size=(n, n)).astype(np.int32))
    D = grid_manhattan(n)
    return Workload("c1_n12_grid_2opt", "2opt", [Instance(F, D, starts(rng, n, k), 0, "c1")], 0)


def c2_dense64(k: int = 128, iters: int = 20000) -> Workload:
    """n=64 asymmetric dense: F, D uniform [0,99]; tabu, k starts x iters, tenure [57,70]."""
    rng = rng_for(2)
    n = 64
    F = uniform_matrix(rng, n, 0, 99)
    D = uniform_matrix(rng, n, 0, 99)
    return Workload("c2_n64_dense_tabu", "tabu", [Instance(F, D, starts(rng, n, k), 2, "c2")], iters)


def c3_instance(rng=None):
    rng = rng if rng is not None else rng_for(3)
    n = 128
    F = symmetrise_upper(sparse_matrix(rng, n, 0.7))
    D = euclid_points(rng, n)
    return F, D


def c3_euclid128_2opt(k: int = 1024) -> Workload:
    """n=128 structured: F 70% zero symmetric, D rounded Euclidean; 2opt from k starts."""
    rng = rng_for(3)
    F, D = c3_instance(rng)
    return Workload("c3_n128_euclid_2opt", "2opt", [Instance(F, D, starts(rng, 128, k), 3, "c3")], 0)


def c3_euclid128_tabu(k: int = 256, iters: int = 10000) -> Workload:
    """Same instance as the 2opt workload; tabu from k starts (drawn after the 2opt starts)."""
    rng = rng_for(3)
    F, D = c3_instance(rng)
    starts(rng, 128, 1024)
    return Workload("c3_n128_euclid_tabu", "tabu", [Instance(F, D, starts(rng, 128, k), 3, "c3")], iters)


def wide_dense512(k: int = 256, iters: int = 2000) -> Workload:
    """n=512 asymmetric dense (beyond the largest QAPLIB sizes): F, D uniform [0,99];
    tabu, k starts x iters, the tenure range of the other tabu workloads."""
    rng = rng_for(6)
    n = 512
    F = uniform_matrix(rng, n, 0, 99)
    D = uniform_matrix(rng, n, 0, 99)
    return Workload("n512_dense_tabu", "tabu", [Instance(F, D, starts(rng, n, k), 6, "wide")], iters)


def stream_dense256(k: int = 256, iters: int = 2000) -> Workload:
    """n=256 asymmetric dense (the largest n of the streamed kernel, as in the serving
    stream's largest requests): F, D uniform [0,99]; tabu, k starts x iters, the tenure
    range of the other tabu workloads."""
    rng = rng_for(7)
    n = 256
    F = uniform_matrix(rng, n, 0, 99)
    D = uniform_matrix(rng, n, 0, 99)
    return Workload("n256_dense_tabu", "tabu", [Instance(F, D, starts(rng, n, k), 7, "stream")], iters)


def c4_batch(m: int = 512, k: int = 8, iters: int = 5000, nmin: int = 20, nmax: int = 150) -> Workload:
    """m instances, n uniform in [nmin, nmax]; even index dense uniform, odd index sparse
    flow (80% zero) with grid-Manhattan distances; tabu with k starts each."""
    rng = rng_for(4)
    insts = []
    for i in range(m):
        n = int(rng.integers(nmin, nmax + 1))
        if i % 2 == 0:
            F = uniform_matrix(rng, n, 0, 99)
            D = uniform_matrix(rng, n, 0, 99)
        else:
            F = sparse_matrix(rng, n, 0.8)
            D = grid_manhattan(n)
        seed = int(rng.integers(0, 2**63 - 1))
        insts.append(Instance(F, D, starts(rng, n, k), seed, "c4_%d" % i))
    return Workload("c4_batched_uneven_tabu", "tabu", insts, iters)


@dataclass
class Request:
    arrival_s: float
    inst: Instance
    iters: int


def c5_stream(count: int = 2000, rate: float = 200.0, nmin: int = 30, nmax: int = 256,
              itmin: int = 2000, itmax: int = 20000) -> list:
    """Poisson arrivals of one-start tabu requests with uneven n and iteration budgets."""
    rng = rng_for(5)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(rng.integers(nmin, nmax + 1))
        sp = float(rng.uniform(0.0, 0.8))
        F = sparse_matrix(rng, n, sp, 0, 99)
        D = uniform_matrix(rng, n, 0, 99)
        it = int(rng.integers(itmin, itmax + 1))
        seed = int(rng.integers(0, 2**63 - 1))
        out.append(Request(t, Instance(F, D, starts(rng, n, 1), seed, "c5_%d" % i), it))
    return out


def random_instance(rng, n, lo=0, hi=99, symmetric=False, diag=False):
    """Small random instance for tests; optional non-zero diagonals."""
    F = rng.integers(lo, hi + 1, size=(n, n)).astype(np.int32)
    D = rng.integers(lo, hi + 1, size=(n, n)).astype(np.int32)
    if symmetric:
        F = np.triu(F) + np.triu(F, 1).T
        D = np.triu(D) + np.triu(D, 1).T
    if not diag:
        np.fill_diagonal(F, 0)
        np.fill_diagonal(D, 0)
    return F.astype(np.int32), D.astype(np.int32)
