"""Sensitivity of tabu to its parameters, as in the paper's study on tai40a and tai40b
(Sec. 6, Figs. 7-9): the number of neighbourhoods explored (iterations), the number of
search instances run in parallel (starts of one launch), and the number of random seeds
(repetitions with fresh starts and tenure draws, the best of k kept, averaged over 8
runs).  Each point reports the quality of the best permutation found and the execution
time of the launch (neighbourhood tables and searches, HIP events on its stream).

QAPLIB's tai40a and tai40b are not in this build, and neither are their best known
costs.  The stand-ins are seeded synthetic instances of the same size and kind:
"a-like", flows and distances uniform in [0, 99]; "b-like", sparse symmetric flows
(70% zeros) and rounded Euclidean distances.  Quality is the gap, in percent, of a
point's best cost over the best cost found for that instance by any run of the sweep,
a long reference run included (1024 starts x 20000 iterations).  The tenure range is the
paper's, [floor(n/10), floor(33n/100)].

    python -m paper_2307_11248_amd.sweep [--out sweep.json]
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import qap
from . import workloads as W

N = 40
ITERS = (50, 100, 200, 400, 800, 1600, 3200, 6400)
INSTANCES = (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024)
SEEDS = (1, 2, 4, 8)
BASE_ITERS = 1000        # iterations of the instance and seed sweeps
BASE_INSTANCES = 256     # search instances of the iteration and seed sweeps
REPEATS = 8              # runs averaged per point of the seed sweep


def stand_ins() -> dict[str, tuple[np.ndarray, np.ndarray]]:
    """The two n = 40 instances: uniform (a-like) and structured (b-like)."""
    rng = np.random.default_rng(4040)
    a = (W.uniform_matrix(rng, N, 0, 99), W.uniform_matrix(rng, N, 0, 99))
    b = (W.symmetrise_upper(W.sparse_matrix(rng, N, 0.7)), W.euclid_points(rng, N))
    return {"a-like": a, "b-like": b}


def gap(best: int, ref: int) -> float:
    """Quality of a best cost against the reference cost, in percent above it."""
    return 100.0 * (best - ref) / ref if ref > 0 else 0.0


def seed_quality(costs: list[list[int]], ref: int) -> float:
    """Seed sweep: costs[r][s] is the best cost of repetition r with seed s; the quality of
    k seeds is the gap of min(costs[r][:k]) averaged over the repetitions."""
    return float(np.mean([gap(min(c), ref) for c in costs]))


class Runner:
    """One instance on the device; run(k, iters, seed) = (best cost, ms) of one launch of
    k tabu searches from seeded random starts."""

    def __init__(self, F: np.ndarray, D: np.ndarray):
        import torch
        self.torch = torch
        self.h = qap.Handle(F, D)
        self.lo, self.hi = W.paper_tenure_range(N)
        self.stream = torch.cuda.Stream()

    def run(self, k: int, iters: int, seed: int) -> tuple[int, float]:
        torch = self.torch
        rng = np.random.default_rng(seed)
        perms = torch.from_numpy(W.starts(rng, N, k)).cuda()
        best = torch.empty(k, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(self.stream):
            e0.record(self.stream)
            self.h.tabu_async(perms, iters, self.lo, self.hi, seed, best, stream=self.stream)
            e1.record(self.stream)
        self.stream.synchronize()
        return int(best.min().item()), float(e0.elapsed_time(e1))

    def close(self):
        self.h.close()


def sweep_instance(name: str, F: np.ndarray, D: np.ndarray, log=sys.stderr) -> dict:
    r = Runner(F, D)
    r.run(64, 100, 1)   # warm-up
    out = {"instance": name, "n": N, "tenure": [r.lo, r.hi]}
    print("[sweep] %s: neighbourhoods" % name, file=log, flush=True)
    out["iterations"] = [(it,) + r.run(BASE_INSTANCES, it, 11) for it in ITERS]
    print("[sweep] %s: search instances" % name, file=log, flush=True)
    out["instances"] = [(k,) + r.run(k, BASE_ITERS, 12) for k in INSTANCES]
    print("[sweep] %s: random seeds" % name, file=log, flush=True)
    runs = [[r.run(BASE_INSTANCES, BASE_ITERS, 1000 * rep + s) for s in range(max(SEEDS))] for rep in range(REPEATS)]
    out["seed_runs"] = [[c for c, _ in row] for row in runs]
    out["seed_ms"] = float(np.mean([ms for row in runs for _, ms in row]))
    print("[sweep] %s: reference" % name, file=log, flush=True)
    out["reference_run"] = r.run(1024, 20000, 99)
    r.close()
    ref = min([c for _, c, _ in out["iterations"]] + [c for _, c, _ in out["instances"]]
              + [c for row in out["seed_runs"] for c in row] + [out["reference_run"][0]])
    out["reference_cost"] = ref
    out["fig_iterations"] = [{"iterations": it, "quality_pct": gap(c, ref), "ms": ms} for it, c, ms in out["iterations"]]
    out["fig_instances"] = [{"instances": k, "quality_pct": gap(c, ref), "ms": ms} for k, c, ms in out["instances"]]
    out["fig_seeds"] = [{"seeds": k, "quality_pct": seed_quality([row[:k] for row in out["seed_runs"]], ref),
                         "ms": k * out["seed_ms"]} for k in SEEDS]
    return out


def markdown(res: list[dict]) -> str:
    lines = []
    for key, col in (("fig_iterations", "iterations"), ("fig_instances", "instances"), ("fig_seeds", "seeds")):
        lines.append("| %s | " % col + " | ".join("%s quality %% | %s ms" % (r["instance"], r["instance"]) for r in res) + " |")
        lines.append("|---|" + "---|---|" * len(res))
        for i in range(len(res[0][key])):
            cells = ["%.2f | %.2f" % (r[key][i]["quality_pct"], r[key][i]["ms"]) for r in res]
            lines.append("| %d | " % res[0][key][i][col] + " | ".join(cells) + " |")
        lines.append("")
    return "\n".join(lines)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=None, help="write the full results as JSON here")
    args = ap.parse_args(argv)
    res = [sweep_instance(name, F, D) for name, (F, D) in stand_ins().items()]
    print(markdown(res))
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(res, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
