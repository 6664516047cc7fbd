#!/usr/bin/env python3
"""Benchmark of the QAP pairwise-exchange hot path on one MI355X.

A step is one pass of the whole hot path over one batch of starts that are already
resident in HBM: reset the working permutations from the starts, build every start's
neighbourhood table, then run every search to completion in one persistent launch.
The default workload is the uneven batch (--workload c4: 512 instances, n from 20 to
150, 8 starts each, 5000 tabu iterations): every start of every instance runs in one
launch of the batched kernels, and the step is a captured HIP graph (reset, tables,
searches) replayed once per step.  Other workloads: c1, c2, c3-2opt, c3-tabu (single
instances), c5 (the serving stream), stream (n = 256, the streamed kernel), wide (n = 512,
the wide streamed kernel).

The roofline is priced in HBM bytes: a swap-delta eval (one neighbourhood entry made
current for one step of one search) is an int32 read and write, 8 bytes, against the
8 TB/s of MI355X's HBM3E; the VALU rate of the same evals is reported beside it.

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

# HBM bytes per launch of the dominant kernel, from rocprofv3 FETCH_SIZE and WRITE_SIZE
# runs scaled by a plain copy's counts (x2 and x1; see the summaries under profiles/),
# valid only for the kernel sources they were taken with.
KERNEL_SOURCES = ["paper_2307_11248_amd/csrc/qap_search.hip", "paper_2307_11248_amd/csrc/qap_internal.h"]
TRAFFIC = {
    "c2_n64_dense_tabu": {"bytes": int((2 * 725.5 + 40.0) * 1024), "sources": "c0b7ca82fda47dff"},
    "c3_n128_euclid_tabu": {"bytes": int((2 * 4415.5 + 144.0) * 1024), "sources": "c0b7ca82fda47dff"},
    # per dispatch, summed over the kernels of one launch (tiles of 2 rows on 128 and 256
    # lanes, of 4 rows on 256, 512 and 768)
    "c4_batched_uneven_tabu": {"bytes": int((2 * (65156.0 + 43345.67 + 8637.87 + 2649.54 + 1970.87)
                                             + (874.563 + 408.78 + 223.25 + 92.625 + 61.5)) * 1024),
                               "sources": "c0b7ca82fda47dff"},
    "n256_dense_tabu": {"bytes": int((2 * 68646900.0 + 67775000.0) * 1024), "sources": "c0b7ca82fda47dff"},
    "n512_dense_tabu": {"bytes": int((2 * 141803000.0 + 266390000.0) * 1024), "sources": "c0b7ca82fda47dff"},
}


def roofline(search_evals, kernel_ms, kernel, traffic, ops_per_eval):
    """HBM roofline of the search phase at 8 B per eval, with the VALU rate beside it."""
    sec = kernel_ms / 1e3
    hbm = BYTES_PER_EVAL * search_evals / sec / 1e9
    valu = ops_per_eval * search_evals / sec / 1e12
    return {"bound": "hbm", "achieved": round(hbm, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(hbm / PEAK_HBM_GBS, 4), "traffic": traffic, "kernel": kernel,
            "kernel_ms": round(kernel_ms, 4), "bytes_per_eval": BYTES_PER_EVAL, "evals_per_launch": search_evals,
            "alu_equivalent": {"achieved": round(valu, 3), "peak": round(PEAK_VALU_TOPS, 3), "unit": "TOP/s",
                               "frac": round(valu / PEAK_VALU_TOPS, 4), "ops_per_eval": ops_per_eval}}


def kernel_digest():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(workload):
    t = TRAFFIC.get(workload)
    return t["bytes"] if t is not None and t["sources"] == kernel_digest() else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4", choices=["c1", "c2", "c3-2opt", "c3-tabu", "c4", "c5", "stream", "wide"])
    ap.add_argument("--tile-rows", type=int, default=0,
                    help="tile rows of the searches (uneven batch: for every instance it fits, else the tuner's)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-launch-per-start comparison")
    ap.add_argument("--cpu-starts", type=int, default=32,
                    help="single instances: oracle starts; uneven batch: at most this many instances "
                         "per oracle leg x 16 (one start each)")
    ap.add_argument("--plain-instances", type=int, default=32,
                    help="uneven batch: instances whose starts are also run one launch per start")
    ap.add_argument("--no-tune", action="store_true", help="uneven batch: the default tile shape for every n")
    ap.add_argument("--chunk-ms", type=float, default=2.0, help="serving: device time per chunk of a search")
    ap.add_argument("--requests", type=int, default=2000, help="serving: requests in the arrival stream")
    ap.add_argument("--tune-cache", default=None, help="uneven batch: JSON cache of tuned tile shapes")
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
    if name == "c4":
        return W.c4_batch()
    if name == "stream":
        return W.stream_dense256()
    if name == "wide":
        return W.wide_dense512()
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


def cpu_baseline_batch(w, gpu_best, gpu_perm, sample):
    """The oracle on a bounded sample of (instance, start) pairs of the uneven batch."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    insts = w.instances
    k = len(insts[0].perms)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    off = np.concatenate([[0], np.cumsum([k * I.n for I in insts])])

    def run(a):
        t, j = a
        I = insts[t]
        lo, hi = w.tenure(I.n)
        return oracle.tabu(I.F, I.D, I.perms[j], w.iters, lo, hi, I.seed, j)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        res = list(ex.map(run, sample))
    dt = time.perf_counter() - t0
    evals = sum(insts[t].n * (insts[t].n - 1) // 2 * (r[2] + 1) for (t, _), r in zip(sample, res))
    exact = all((gpu_perm[off[t] + j * insts[t].n: off[t] + (j + 1) * insts[t].n] == r[0]).all()
                and gpu_best[t * k + j] == r[1] for (t, j), r in zip(sample, res))
    return {"value": evals / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": "%d (instance, start) pairs of the uneven batch, one start per instance spread over "
                      "the batch, run to completion (%.1f s wall)" % (len(sample), dt)}, exact


def run_batch(args, w):
    import torch
    from paper_2307_11248_amd import qap
    insts = w.instances
    m, k = len(insts), len(insts[0].perms)
    hs = [qap.Handle(I.F, I.D) for I in insts]
    lo = [w.tenure(I.n)[0] for I in insts]
    hi = [w.tenure(I.n)[1] for I in insts]
    seeds = [I.seed for I in insts]
    tune_s, rows_hist = None, None
    if not args.no_tune:
        from paper_2307_11248_amd.autotune import TileCache
        t0 = time.perf_counter()
        cache = TileCache(args.tune_cache)
        rows = cache.apply_all(hs, "batch")
        cache.save()
        tune_s = time.perf_counter() - t0
        if args.tile_rows:
            for t, h in enumerate(hs):
                try:
                    h.set_tile_rows("batch", args.tile_rows)
                    rows[t] = args.tile_rows
                except qap.QapError:
                    pass
        rows_hist = {str(r): rows.count(r) for r in sorted(set(rows))}
    b = qap.Batch(hs, [k] * m, w.iters, lo, hi, seeds)
    stream = torch.cuda.Stream()
    starts = torch.from_numpy(np.concatenate([I.perms.reshape(-1) for I in insts])).cuda()
    work = torch.empty_like(starts)
    best = torch.empty(m * k, dtype=torch.int64, device="cuda")
    done = torch.empty(m * k, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()

    # kernel durations: the same three launches, eagerly, bracketed by events on their stream
    ev = []
    for rep in range(args.warmup + args.steps):
        with torch.cuda.stream(stream):
            work.copy_(starts)
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(stream)
            b.tables_async(work, stream=stream)
            e[1].record(stream)
            b.search_async(work, best, done, stream=stream)
            e[2].record(stream)
        if rep >= args.warmup:
            ev.append(e)
    torch.cuda.synchronize()
    table_ms = float(np.mean([a.elapsed_time(c) for a, c, _ in ev]))
    search_ms = float(np.mean([c.elapsed_time(d) for _, c, d in ev]))
    eager_p, eager_c = work.cpu().numpy(), best.cpu().numpy()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        work.copy_(starts)
        b.run_async(work, best, done, stream=stream)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    # the search phase as the graph runs it: the same back-to-back replays, bracketed by two
    # events on the replay stream (after the timed loop), less the table kernel's own time
    # from the eager runs
    rs = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(rs)
    for _ in range(args.steps):
        g.replay()
    e1.record(rs)
    torch.cuda.synchronize()
    replay_ms = e0.elapsed_time(e1) / args.steps
    eager_search_ms = search_ms
    search_ms = replay_ms - table_ms
    gpu_perm, gpu_best = work.cpu().numpy(), best.cpu().numpy()
    moves = done.cpu().numpy().astype(np.int64)
    assert (gpu_perm == eager_p).all() and (gpu_best == eager_c).all(), "graph replay differs from eager run"
    ms = np.repeat([I.n * (I.n - 1) // 2 for I in insts], k).astype(np.int64)
    off = np.concatenate([[0], np.cumsum([k * I.n for I in insts])])
    for t, I in enumerate(insts):
        assert (hs[t].cost(gpu_perm[off[t]:off[t + 1]].reshape(k, I.n)) == gpu_best[t * k:(t + 1) * k]).all()
    evals_step = int((ms * (moves + 1)).sum())
    search_evals = int((ms * moves).sum())
    value = evals_step / (ms_step / 1e3)
    # the search phase: one batch_group_kernel dispatch per tile-shape variant, forked onto
    # side streams and joined back; the events bracket the fork and the join
    roof = roofline(search_evals, search_ms, "batch_group_kernel (search phase: %d variant dispatches on the "
                    "graph's lanes; replay time less the table kernel)" % b.groups(), traffic_for(w.name),
                    VALU_PER_EVAL["tabu"])
    roof["replay_ms"] = round(replay_ms, 4)
    roof["eager_search_ms"] = round(eager_search_ms, 4)
    ns = [I.n for I in insts]
    out = {"metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": w.name, "instances": m, "n_range": [min(ns), max(ns)], "starts_per_instance": k,
                      "iters": w.iters, "tenure": "[0.9n, 1.1n]", "graph": True,
                      "tile_rows_per_instance": rows_hist, "tuning_s": tune_s,
                      "searches_per_variant": dict(zip(["r2_512", "r4_512", "r8_512", "stream_512", "r2_128",
                                                        "r2_256", "r4_256", "r4_768", "wide_512"],
                                                       map(int, b.groups(counts=True)[1])))},
           "solves_per_s": m * k / (ms_step / 1e3), "table_kernel_ms": table_ms, "roofline": roof}

    if not args.no_plain:
        batched_solves = m * k / (ms_step / 1e3)
        # (1) the plain path: one launch per start, back to back on one stream, on the
        #     starts of a sample of instances spread over the batch (the whole batch
        #     would take about a minute this way)
        pi = list(range(0, m, max(1, m // args.plain_instances)))[:args.plain_instances]
        pw = starts.clone()
        pb = torch.empty(m * k, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            for t in pi:
                I = insts[t]
                hs[t].tabu_async(pw[off[t]:off[t + 1]].view(k, I.n), w.iters, lo[t], hi[t], I.seed,
                                 pb[t * k:(t + 1) * k], None, plain=True, stream=stream)
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t0
        pw_h, pb_h = pw.cpu().numpy(), pb.cpu().numpy()
        same = all((pb_h[t * k:(t + 1) * k] == gpu_best[t * k:(t + 1) * k]).all()
                   and (pw_h[off[t]:off[t + 1]] == gpu_perm[off[t]:off[t + 1]]).all() for t in pi)
        out["plain"] = {"solves_per_s": len(pi) * k / pdt, "speedup_batched_vs_plain": batched_solves / (len(pi) * k / pdt),
                        "identical_costs": bool(same),
                        "sample": "one launch per start for the %d starts of %d instances spread over the batch"
                                  % (len(pi) * k, len(pi))}
        # (2) one launch per instance (k blocks each), the whole batch
        pw = starts.clone()
        pb = torch.empty(m * k, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            for t, I in enumerate(insts):
                hs[t].tabu_async(pw[off[t]:off[t + 1]].view(k, I.n), w.iters, lo[t], hi[t], I.seed,
                                 pb[t * k:(t + 1) * k], None, stream=stream)
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t0
        out["per_instance_launches"] = {
            "solves_per_s": m * k / pdt, "speedup_batched": batched_solves / (m * k / pdt),
            "identical_costs": bool((pb.cpu().numpy() == gpu_best).all() and (pw.cpu().numpy() == gpu_perm).all())}

    if not args.no_cpu:
        # one start of every instance, up to 16 x --cpu-starts of them (the default covers all
        # 512 instances, every tile-shape variant, about a tenth of the batch's evals)
        cap = 16 * args.cpu_starts
        step = max(1, -(-m // cap))
        sample = [(t, t % k) for t in range(0, m, step)][:cap]
        cb, exact = cpu_baseline_batch(w, gpu_best, gpu_perm, sample)
        out["cpu_baseline"] = cb
        out["bit_exact_sample"] = exact
    b.close()
    for h in hs:
        h.close()
    print(json.dumps(out), flush=True)


def run_serve(args):
    """The serving stream: Poisson arrivals replayed in real time into the server."""
    import torch
    from paper_2307_11248_amd import qap
    from paper_2307_11248_amd import workloads as W
    reqs = W.c5_stream(count=args.requests)
    N = len(reqs)
    srv = qap.Server(8 << 30, 256, args.chunk_ms)
    # warm-up: a few requests through the same server (kernels loaded, pool touched)
    for r in reqs[:args.warmup * 4]:
        lo, hi = W.tabu_tenure_range(r.inst.n)
        t = srv.submit(r.inst.F, r.inst.D, r.inst.perms[0], 200, lo, hi, r.inst.seed)
        while srv.result(t) is None:
            srv.step()
    torch.cuda.synchronize()
    tickets, outstanding, lat, results = {}, {}, {}, {}
    i = 0
    t0 = time.perf_counter()
    while len(results) < N:
        now = time.perf_counter() - t0
        while i < N and reqs[i].arrival_s <= now:
            r = reqs[i]
            lo, hi = W.tabu_tenure_range(r.inst.n)
            t = srv.submit(r.inst.F, r.inst.D, r.inst.perms[0], r.iters, lo, hi, r.inst.seed)
            tickets[t] = outstanding[t] = i
            i += 1
        if len(tickets) == len(results):          # idle: wait for the next arrival
            if i < N:
                time.sleep(max(0.0, reqs[i].arrival_s - (time.perf_counter() - t0)))
            continue
        f, _, _ = srv.step()
        t_done = time.perf_counter() - t0
        if f:
            for t in [t for t in outstanding]:
                res = srv.result(t)
                if res is not None:
                    j = outstanding.pop(t)
                    results[j] = res
                    lat[j] = (t_done - reqs[j].arrival_s) * 1e3
    wall = time.perf_counter() - t0
    stats = srv.stats()
    ms = np.array([r.inst.n * (r.inst.n - 1) // 2 for r in reqs], dtype=np.int64)
    moves = np.array([results[j][2] for j in range(N)], dtype=np.int64)
    evals = int((ms * (moves + 1)).sum())
    L = np.array([lat[j] for j in range(N)])
    # a sample of requests run alone (qap_tabu, start id 0) must give the same results
    same = True
    for j in range(0, N, max(1, N // 8)):
        r = reqs[j]
        lo, hi = W.tabu_tenure_range(r.inst.n)
        with qap.Handle(r.inst.F, r.inst.D) as h:
            bp, bc, bd = h.tabu(r.inst.perms, r.iters, lo, hi, r.inst.seed)
        same = same and bool((bp[0] == results[j][0]).all() and bc[0] == results[j][1] and bd[0] == results[j][2])
    ns = [r.inst.n for r in reqs]
    out = {"metric": METRIC, "value": evals / wall, "unit": "evals/s", "n_gpus": 1, "steps": 1,
           "warmup": args.warmup, "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "c5_serving_stream", "requests": N, "rate_per_s": 200.0,
                      "n_range": [min(ns), max(ns)], "iters_range": [min(r.iters for r in reqs),
                                                                     max(r.iters for r in reqs)],
                      "chunk_ms": args.chunk_ms, "max_active": 256, "pool_bytes": 8 << 30},
           "solves_per_s": N / wall,
           "latency_ms": {"p50": float(np.percentile(L, 50)), "p99": float(np.percentile(L, 99)),
                          "mean": float(L.mean()), "max": float(L.max())},
           "server": stats, "identical_alone_sample": same}
    if not args.no_cpu:
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        sample = list(range(0, N, max(1, N // args.cpu_starts)))[:args.cpu_starts]

        def one(j):
            r = reqs[j]
            lo, hi = W.tabu_tenure_range(r.inst.n)
            return oracle.tabu(r.inst.F, r.inst.D, r.inst.perms[0], r.iters, lo, hi, r.inst.seed, 0)

        t1 = time.perf_counter()
        with ThreadPoolExecutor(cores) as ex:
            cres = list(ex.map(one, sample))
        cdt = time.perf_counter() - t1
        cev = sum(int(ms[j]) * (c[2] + 1) for j, c in zip(sample, cres))
        out["cpu_baseline"] = {"value": cev / cdt, "unit": "evals/s", "cores": cores, "kind": "oracle",
                               "sample": "%d requests of the stream, each run to its iteration budget "
                                         "(%.1f s wall)" % (len(sample), cdt)}
        out["bit_exact_sample"] = all((results[j][0] == c[0]).all() and results[j][1] == c[1]
                                      for j, c in zip(sample, cres))
    srv.close()
    print(json.dumps(out), flush=True)


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
    if args.workload == "c5":
        return run_serve(args)
    w = load_workload(args.workload)
    if len(w.instances) > 1:
        return run_batch(args, w)
    I = w.instances[0]
    n, k = I.n, len(I.perms)
    m = n * (n - 1) // 2
    lo, hi = w.tenure(n)
    h = qap.Handle(I.F, I.D)
    algo = w.algo
    if args.tile_rows:
        h.set_tile_rows(algo, args.tile_rows)
    rows, lanes = h.launch_tile_rows(algo, k)   # the shape the launch of all k starts uses

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
    kname = ("search_kernel<%d,%s>" % (rows, "true" if algo == "tabu" else "false") if rows > 0 else
             "stream_kernel<%s,false,%s>" % ("true" if algo == "tabu" else "false",
                                             "true" if n > 256 else "false"))
    roof = roofline(search_evals, search_ms, kname, traffic_for(w.name), VALU_PER_EVAL[algo])

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
