#!/usr/bin/env python3
"""Benchmark of the QAP pairwise-exchange hot path on one MI355X.

A step is one pass of the whole hot path over one batch of starts that are already
resident in HBM: reset the working permutations from the starts, build every start's
neighbourhood table, then run every search to completion in one persistent launch.

Prints one JSON line (see the keys below).  --gpus N with N > 1 is refused: this build
runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "swap-delta evals/sec; batched tabu solves/sec vs plain, bit-exact costs"
PEAK_HBM_GBS = 8000.0
# VALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# VALU lane-instructions one neighbourhood entry needs per step on gfx950:
# update (two v_pk_sub_i16, one v_dot2_i32_i16) + admissible minimum (two compares for
# tabu state and aspiration, one compare and two selects for the running minimum)
VALU_PER_EVAL = {"tabu": 8, "2opt": 6}
BYTES_PER_EVAL = 8   # an int32 delta read and written per entry per step if kept in HBM


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3-2opt", "c3-tabu"])
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-launch-per-start comparison")
    ap.add_argument("--cpu-starts", type=int, default=32)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (to scale HBM byte counters)")
    return ap.parse_args()


def load_workload(name):
    from paper_2307_11248_amd import workloads as W
    if name == "c1":
        return W.c1_grid12()
    if name == "c2":
        return W.c2_dense64()
    if name == "c3-2opt":
        return W.c3_euclid128_2opt()
    return W.c3_euclid128_tabu()


def cpu_baseline(w, gpu_best, gpu_perm, nstarts):
    """The oracle, as it is, on a bounded sample of the same workload, on every host core."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    I = w.instances[0]
    n = I.n
    m = n * (n - 1) // 2
    idx = list(range(min(nstarts, len(I.perms))))
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    lo, hi = w.tenure(n)

    def run(j):
        if w.algo == "tabu":
            bp, bc, done, _ = oracle.tabu(I.F, I.D, I.perms[j], w.iters, lo, hi, I.seed, j)
            return bp, bc, done
        q, c, st, _ = oracle.two_opt(I.F, I.D, I.perms[j])
        return q, c, st

    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        res = list(ex.map(run, idx))
    dt = time.perf_counter() - t0
    if w.algo == "tabu":
        evals = sum(m * (r[2] + 1) for r in res)
    else:
        evals = sum(m * (r[2] + 1) for r in res)
    exact = all((gpu_perm[j] == r[0]).all() and gpu_best[j] == r[1] for j, r in zip(idx, res))
    return {"value": evals / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": "%d of %d starts of the same workload, run to completion (%.1f s wall)"
                      % (len(idx), len(I.perms), dt)}, exact


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2307_11248_amd import qap

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": nbytes, "copy_calibration_bytes_written": nbytes}))
        return
    w = load_workload(args.workload)
    I = w.instances[0]
    n, k = I.n, len(I.perms)
    m = n * (n - 1) // 2
    lo, hi = w.tenure(n)
    h = qap.Handle(I.F, I.D)
    algo = w.algo
    if args.tile_rows:
        h.set_tile_rows(algo, args.tile_rows)
    rows, lanes = h.tile_rows(algo)

    stream = torch.cuda.Stream()
    starts = torch.from_numpy(I.perms).cuda()
    work = torch.empty_like(starts)
    table = torch.empty((k, m), dtype=torch.int32, device="cuda")
    best = torch.empty(k, dtype=torch.int64, device="cuda")
    done = torch.empty(k, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()

    ev = []

    def step(record):
        with torch.cuda.stream(stream):
            work.copy_(starts)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e2 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            h.delta_table_async(work, table, stream=stream)
            e1.record(stream)
            if algo == "tabu":
                h.tabu_with_table_async(work, table, w.iters, lo, hi, I.seed, best, done, stream=stream)
            else:
                h.two_opt_with_table_async(work, table, best, done, max_iters=w.iters, stream=stream)
            e2.record(stream)
            if record:
                ev.append((e0, e1, e2))

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    table_ms = float(np.mean([a.elapsed_time(b) for a, b, c in ev]))
    search_ms = float(np.mean([b.elapsed_time(c) for a, b, c in ev]))
    moves = done.cpu().numpy().astype(np.int64)
    evals_step = int((moves + 1).sum()) * m
    value = evals_step / (ms_step / 1e3)
    solves = k / (ms_step / 1e3)
    gpu_best = best.cpu().numpy()
    gpu_perm = work.cpu().numpy()
    assert (h.cost(gpu_perm) == gpu_best).all(), "returned costs are not Eq. (1) of the returned permutations"

    search_evals = int(moves.sum()) * m
    valu = VALU_PER_EVAL[algo] * search_evals / (search_ms / 1e3) / 1e12
    roof = {"bound": "alu", "achieved": round(valu, 3), "peak": round(PEAK_VALU_TOPS, 3), "unit": "TOP/s",
            "frac": round(valu / PEAK_VALU_TOPS, 4), "traffic": None,
            "kernel": "search_kernel<%d,%s>" % (rows, "true" if algo == "tabu" else "false"),
            "kernel_ms": round(search_ms, 4),
            "ops_per_eval": VALU_PER_EVAL[algo],
            "hbm_equivalent": {"achieved": round(BYTES_PER_EVAL * search_evals / (search_ms / 1e3) / 1e9, 1),
                               "peak": PEAK_HBM_GBS, "unit": "GB/s",
                               "frac": round(BYTES_PER_EVAL * search_evals / (search_ms / 1e3) / 1e9
                                             / PEAK_HBM_GBS, 4)}}

    out = {"metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": w.name, "n": n, "starts": k, "iters": w.iters,
                      "tenure": [lo, hi] if algo == "tabu" else None, "tile_rows": rows,
                      "lanes_per_search": lanes},
           "solves_per_s": solves, "table_kernel_ms": table_ms, "roofline": roof}

    if algo == "tabu" and not args.no_plain:
        pw = starts.clone()
        pb = torch.empty(k, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            h.tabu_async(pw, w.iters, lo, hi, I.seed, pb, None, plain=True, stream=stream)
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t0
        out["plain"] = {"solves_per_s": k / pdt, "speedup_batched_vs_plain": (k / pdt and solves / (k / pdt)),
                        "identical_costs": bool((pb.cpu().numpy() == gpu_best).all()
                                                and (pw.cpu().numpy() == gpu_perm).all())}

    if not args.no_cpu:
        cb, exact = cpu_baseline(w, gpu_best, gpu_perm, args.cpu_starts)
        out["cpu_baseline"] = cb
        out["bit_exact_sample"] = exact
    h.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
