"""Benchmark of the Boolean-matrix miner on one MI355X.

One step = the whole hot path on one synthetic database already resident in
HBM: matrix construction from the CSR transaction list (bm_build), single-item
supports, pair supports (A^T A on MFMA: scaled FP4 (e2m1) operands with exact
FP32 sums by default, int8 on request), the recursive extension of frequent
prefixes (masked Gram on MFMA for large prefix classes, subset counting or
AND+popcount for small ones), and the canonical-order result (bm_mine).
Prints one JSON line.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--workload 3]

value = candidate supports counted per second of step wall time (pairs of
frequent items plus every longer candidate; the two parts are reported
separately in config), with the step's wall time in ms_per_step.  `roofline`
describes the kernel with the largest total time, measured with hipEvents
recorded by the library on the call's stream.  After the timed steps, more
steps write a 2 GiB scratch buffer between build and mine so that the mine
call starts with L2 and the Infinity Cache holding none of the matrix; their
kernel rates are reported as `cache_cold`.  By default the batched workload
(256 databases: plain per-database, batched, batched + learned order) and
the T40-style workload (plain and learned subtree order) are also run and
reported under `secondary`.
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

HBM_PEAK_GBS = 8000.0
# dense MFMA peaks of MI355X by operand type (TOP/s)
MFMA_PEAK_TOPS = {"int8": 5000.0, "fp4": 10100.0}
# contractions priced against the MFMA peak of their operand type: algorithmic
# ops = 2 n per candidate pair (one AND, one add per transaction)
MFMA_KERNELS = {
    "gram_mfma": "k_gram_mfma (MFMA Gram of a prefix class, 128x128 tiles)",
    "gram_mfma_big": "k_gram_mfma_big (MFMA Gram of a big prefix class, 256x256 tiles, one workgroup per CU)",
    "gram_small": "k_gram_small (MFMA Gram of a mid-size class, 32x32 tiles, one wave per task)",
}
# streaming kernels priced against HBM: algorithmic bytes = column words read
HBM_KERNELS = {
    "andpop": "k_andpop (AND+popcount of a prefix class, LDS-blocked)",
    "andpop_reg": "k_andpop_reg (AND+popcount of a small prefix class in registers)",
    "dfs": "small-class subtrees: k_subset_count + k_subset_emit (every subset of a class's "
           "children counted over word ranges; long columns) or k_dfs (depth-first from a work "
           "queue; short columns)",
}

WORKLOADS = {
    1: "basket_zipf 10,000 tx x 169 items, minsup 1% (100)",
    2: "quest T10I4D100K-style 100,000 tx x 1,000 items, minsup 0.25% (250)",
    3: "dense_planted 1,000,000 tx x 4,096 items, 500 planted 6-item patterns, minsup 1% (10,000)",
    4: "batch of 256 quest-style databases (1k-200k tx log-uniform, 50-2,000 items, mean length "
       "5-20, minsup 0.5-5%)",
    5: "quest T40I10D1M-style 1,000,000 tx x 2,000 items, minsup 0.5% (5,000)",
}


def _host_cpu():
    """Host cores available to this process and the CPU model (from /proc/cpuinfo)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return avail, os.cpu_count() or avail, model


def cpu_baseline(db, target_s: float = 12.0, single_s: float = 4.0) -> dict:
    """The C++ oracle as it stands, on a bounded sample of the same workload:
    the subtrees of the first k frequent items (all itemsets whose smallest
    item is one of them), k grown until one run takes about `target_s`
    (at least 10 s of CPU work unless the whole workload finishes sooner),
    on every available host core up to 16; then a smaller sample on one
    thread (about `single_s`)."""
    from oracle import cpp as ocpp
    avail, online, model = _host_cpu()
    threads = max(1, min(16, avail))
    o = ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m)
    m1 = len(o.frequent_items(db.minsup))

    def grow(nthreads, goal, floor):
        k = max(1, min(m1, nthreads))
        dt, cands, sets_ = o.time_sample(db.minsup, 0, k, nthreads)
        for _ in range(8):
            if dt >= floor or k >= m1:
                break
            # subtree costs fall with the item index, so extrapolate generously
            k = min(m1, max(k + 1, int(k * goal / max(dt, 1e-3))))
            dt, cands, sets_ = o.time_sample(db.minsup, 0, k, nthreads)
        return k, dt, cands, sets_

    k, dt, cands, sets_ = grow(threads, target_s, 10.0)
    k1, dt1, cands1, _ = grow(1, single_s, 3.0)
    return {
        "value": cands / dt if dt > 0 else None,
        "unit": "candidate supports/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"C++ sorted-tid-vector oracle, {threads} threads, subtrees of the first {k} of "
                  f"{m1} frequent items: {cands} candidate supports, {sets_} frequent sets in {dt:.2f} s",
        "seconds": round(dt, 3),
        "host": {"cpu_model": model, "cores_available": avail, "cores_online": online},
        "single_thread": {"value": cands1 / dt1 if dt1 > 0 else None, "seconds": round(dt1, 3),
                          "sample": f"1 thread, subtrees of the first {k1} frequent items: "
                                    f"{cands1} candidate supports"},
    }


def _kernel_table(stats, steps):
    names = list(stats[0]["kernel_ms"])
    ms = {k: sum(s["kernel_ms"][k] for s in stats) for k in names}
    launches = {k: sum(s["kernel_launches"][k] for s in stats) for k in names}
    kernels = {}
    for k in names:
        if launches[k] == 0:
            continue
        per = ms[k] / launches[k]
        by = sum(s["kernel_bytes"][k] for s in stats) / launches[k]
        op = sum(s["kernel_ops"][k] for s in stats) / launches[k]
        kernels[k] = {"ms_per_step": round(ms[k] / steps, 4), "launches_per_step":
                      launches[k] / steps, "avg_launch_ms": round(per, 4)}
        if k in MFMA_KERNELS:
            kernels[k]["achieved_TOPs"] = round(op / (per * 1e-3) / 1e12, 2)
            kernels[k]["algorithmic_ops_per_launch"] = op
        if k in HBM_KERNELS:
            kernels[k]["achieved_GBs"] = round(by / (per * 1e-3) / 1e9, 1)
            kernels[k]["algorithmic_bytes_per_launch"] = by
    return kernels, ms


DTYPE = {"fp4": "u64 bitsets; fp4 (e2m1) MFMA, fp32 accumulate (exact: counts < 2^24 per task)",
         "int8": "u64 bitsets; int8 MFMA, int32 accumulate"}

# HBM traffic per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes (scaled by
# the copy calibration), valid only while the kernel's source is unchanged:
# (workload, kernel, form) -> (source file, its sha256, bytes per launch).
TRAFFIC = {
    # dense_planted 1M x 4,096, cache-cold mine (profiles/dense_planted_1M_hbm_traffic.md); the
    # Gram entries also hash the task generation, which decides the tiles a launch computes
    (3, "gram_mfma", "fp4"): (("k_gram_mfma.hip", "gram_fp4.hpp", "internal.hpp", "k_levels.hip", "levels.hpp"), "b5b0d612e6a4a81393ecb9db6a59bb527a591ef697d7322eaf29f9e57f7b5edd", 4638.5e6),
    (3, "gram_small", "fp4"): (("k_gram_small.hip", "internal.hpp", "k_levels.hip", "levels.hpp"), "12aff1a997e66c468caaba250b2bd88f261c9f6dedc5743b57be77b9ead886b4", 268.2e6),
    (3, "dfs", "fp4"): (("k_subsets.hip", "internal.hpp"), "7733ae4634918b5e502294cd009d3e1dd5e305d1f82bd7f37077fffdff1370c0", 756.7e6),
    # Quest T40-style 1M x 2,000, cache-cold mine (profiles/quest_t40_1M_hbm_traffic.md)
    (5, "gram_mfma", "fp4"): (("k_gram_mfma.hip", "gram_fp4.hpp", "internal.hpp", "k_levels.hip", "levels.hpp"), "b5b0d612e6a4a81393ecb9db6a59bb527a591ef697d7322eaf29f9e57f7b5edd", 2569.1e6),
    (5, "gram_small", "fp4"): (("k_gram_small.hip", "internal.hpp", "k_levels.hip", "levels.hpp"), "12aff1a997e66c468caaba250b2bd88f261c9f6dedc5743b57be77b9ead886b4", 217.4e6),
    (5, "dfs", "fp4"): (("k_subsets.hip", "internal.hpp"), "7733ae4634918b5e502294cd009d3e1dd5e305d1f82bd7f37077fffdff1370c0", 347.7e6),
}
WORKLOAD = None


def traffic_of(kernel: str, form: str):
    rec = TRAFFIC.get((WORKLOAD, kernel, form))
    if rec is None:
        return None
    import hashlib
    files = rec[0] if isinstance(rec[0], tuple) else (rec[0],)
    h = hashlib.sha256()
    for name in files:  # the kernel's sources as measured
        with open(os.path.join(ROOT, "paper_2412_19420_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec[1]:
        return None
    return rec[2]


def _roofline(kernels, ms, form):
    dom = max((k for k in kernels if k in MFMA_KERNELS or k in HBM_KERNELS), key=lambda k: ms[k],
              default=None)
    if dom in MFMA_KERNELS:
        a = kernels[dom]["achieved_TOPs"]
        peak = MFMA_PEAK_TOPS[form]
        return {"bound": "mfma", "kernel": f"{MFMA_KERNELS[dom]}, {form} operands",
                "achieved": a, "peak": peak, "unit": "TOP/s",
                "frac": round(a / peak, 4), "traffic": traffic_of(dom, form)}
    if dom is not None:
        a = kernels[dom]["achieved_GBs"]
        return {"bound": "hbm", "kernel": HBM_KERNELS[dom], "achieved": a, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(a / HBM_PEAK_GBS, 4), "traffic": traffic_of(dom, form)}
    return None


def _makespan(costs, order, workers):
    """Greedy list scheduling, as the persistent queue assigns tasks."""
    import heapq
    heap = [0.0] * workers
    for t in order:
        heapq.heapreplace(heap, heap[0] + costs[t])
    return float(max(heap))


def run_batched(args, bm, torch, dev, steps=None, warmup=None):
    """The batched workload: 256 databases per step, mined four ways on the same
    device-resident inputs -- one plain level-synchronous call per database
    (the plain GPU miner), one batched level-synchronous call, one batched call
    with the depth-first phase in queue order, and one batched call whose
    subtree queue is ordered by the cost model.  The model is trained first, on
    the GPU, on traces of 64 held-out databases of the same distribution."""
    import gen
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    t0 = time.time()
    dbs = gen.make_config(4)
    held = [gen.batch_db(k) for k in range(256, 320)]
    print(f"# 256 + 64 databases generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    dev_in = [(torch.from_numpy(d.row_ptr.astype(np.uint64)).to(dev),
               torch.from_numpy(d.col_idx.astype(np.uint32)).to(dev)) for d in dbs]
    ms_list = [d.minsup for d in dbs]

    def build_each(items, src):
        return [bm.bm_build(rp, ci, d.n, d.m, stream=stream) for d, (rp, ci) in zip(items, src)]

    def build_batch(items, src):
        return bm.bm_build_batch([(rp, ci, d.n, d.m) for d, (rp, ci) in zip(items, src)],
                                 stream=stream)

    # cost model: trained on the GPU from traces of the held-out databases
    hh = build_batch(held, [(torch.from_numpy(d.row_ptr.astype(np.uint64)).to(dev),
                           torch.from_numpy(d.col_idx.astype(np.uint32)).to(dev)) for d in held])
    tr = bm.bm_mine_batch(hh, [d.minsup for d in held], opts=bm.options(bm.FLAG_TRACE),
                          stream=stream)
    f, y = tr[0].trace()
    model = bm.Model(seed=1)
    t1 = time.time()
    loss = model.train(f, y, epochs=40, lr=3e-3, batch=256, stream=stream)
    print(f"# cost model: {len(y)} traced tasks, final loss {loss:.4f}, trained in "
          f"{time.time() - t1:.2f} s", file=sys.stderr, flush=True)
    del tr, hh

    timing = 0 if args.no_timing else bm.FLAG_TIMING | bm.FLAG_TIMING_MAIN
    o_ls = bm.options(timing | bm.FLAG_LEVELSYNC)
    o_dfs = bm.options(timing | bm.FLAG_DEPTH_FIRST)
    # mode: (build, mine); the plain miner builds and mines one database per call
    modes = {
        "plain_per_db": (build_each, lambda hs: [bm.bm_mine_ex(h, m, o_ls, stream=stream)
                                                 for h, m in zip(hs, ms_list)]),
        "batched_levelsync": (build_batch, lambda hs: bm.bm_mine_batch(hs, ms_list, opts=o_ls,
                                                                       stream=stream)),
        "batched_depth_first": (build_batch, lambda hs: bm.bm_mine_batch(hs, ms_list, opts=o_dfs,
                                                                         stream=stream)),
        "batched_learned": (build_batch, lambda hs: bm.bm_mine_batch(hs, ms_list, model=model,
                                                                     opts=o_dfs, stream=stream)),
    }
    # what the learned order buys, independent of timing noise: the realised
    # subtree costs of this batch's depth-first queue list-scheduled over the
    # kernel's workgroups in plain and in learned order (untimed)
    hs = build_batch(dbs, dev_in)
    f, y = bm.bm_mine_batch(hs, ms_list, opts=bm.options(bm.FLAG_TRACE), stream=stream)[0].trace()
    cost = np.exp2(y.astype(np.float64)) - 1
    pred = model.predict(f, stream=stream).astype(np.float64)
    workers = torch.cuda.get_device_properties(0).multi_processor_count * 8
    sched_sim = {
        "tasks": int(len(cost)), "workers": workers,
        "plain_makespan_words": _makespan(cost, range(len(cost)), workers),
        "learned_makespan_words": _makespan(cost, np.argsort(-pred, kind="stable"), workers),
        "true_cost_lpt_makespan_words": _makespan(cost, np.argsort(-cost, kind="stable"), workers),
    }
    del hs

    # identical output in every mode (checked once, untimed)
    ref = [r.arrays() for r in modes["plain_per_db"][1](build_each(dbs, dev_in))]
    for name in list(modes)[1:]:
        build, fn = modes[name]
        got = fn(build(dbs, dev_in))
        for a, b in zip(ref, got):
            assert all(np.array_equal(x, y) for x, y in zip(a, b.arrays())), name
    print("# all modes give identical results", file=sys.stderr, flush=True)

    res = {}
    for name, (build, fn) in modes.items():
        for _ in range(warmup):
            fn(build(dbs, dev_in))
        torch.cuda.synchronize()
        stats = []
        t_start = time.perf_counter()
        build_s = 0.0
        kept = []
        for i in range(steps):
            tb = time.perf_counter()
            hs = build(dbs, dev_in)
            torch.cuda.synchronize()
            build_s += time.perf_counter() - tb
            rs = fn(hs)
            torch.cuda.synchronize()
            kept.append(rs)
            del hs, rs
        total = time.perf_counter() - t_start
        # statistics are read after the timed region
        for rs in kept:
            stats.append(rs[0].stats() if name != "plain_per_db" else None)
            if name == "plain_per_db":
                cand = sum(r.stats()["candidates_total"] for r in rs)
            else:
                cand = rs[0].stats()["candidates_total"]
        del kept
        res[name] = {"ms_per_step": round(1e3 * total / steps, 3),
                     "build_ms": round(1e3 * build_s / steps, 3),
                     "mine_ms": round(1e3 * (total - build_s) / steps, 3),
                     "candidates": cand, "stats": stats}
        print(f"# {name}: {res[name]['ms_per_step']} ms/step (mine {res[name]['mine_ms']} ms)",
              file=sys.stderr, flush=True)

    best = res["batched_learned"]
    kernels, kms = (_kernel_table(best["stats"], steps) if not args.no_timing else ({}, {}))
    st = best["stats"][-1]
    out = {
        "metric": "candidate supports counted/s + mine wall time at minsup; % of HBM peak",
        "value": round(best["candidates"] / (best["ms_per_step"] * 1e-3), 1),
        "unit": "candidate supports/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": best["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[st["mfma_form"]],
        "data": "synthetic (seeded generator, see DESIGN.md)",
        "config": {"workload": WORKLOADS[4], "databases": len(dbs), "candidates": best["candidates"],
                   "dfs_tasks": st["dfs_tasks"], "host_syncs": st["host_syncs"],
                   "modes": {k: {kk: vv for kk, vv in v.items() if kk != "stats"}
                             for k, v in res.items()},
                   "learned_vs_plain_speedup": round(res["plain_per_db"]["ms_per_step"] /
                                                     best["ms_per_step"], 3),
                   "learned_vs_batched_depth_first": round(res["batched_depth_first"]["mine_ms"] /
                                                           best["mine_ms"], 3),
                   "queue_makespan_simulation": sched_sim,
                   "kernels": kernels},
        "roofline": _roofline(kernels, kms, st["mfma_form"]) if kernels else None,
    }
    return out


def _single_opts(bm, args, flags, **over):
    kw = dict(mfma_min_children=args.mfma_min_children, mfma_big_children=args.mfma_big_children,
              split_words=args.split_words, shuffle_seed=args.shuffle, dfs_threads=args.dfs_threads,
              dfs_max_words=args.dfs_max_words)
    kw.update(over)
    return bm.options(flags=flags, **kw)


def run_single(args, bm, torch, dev, workload, steps, warmup, sched="none", extra_flags=0,
               dfs_max_words=None, cold_steps=3, quiet=False):
    """One database per step: bm_build + bm_mine on device-resident CSR.
    Returns the bench record (without the CPU baseline)."""
    import gen
    t0 = time.time()
    db = gen.make_config(workload)
    print(f"# workload {workload}: {db.name} n={db.n} m={db.m} nnz={db.nnz} minsup={db.minsup} "
          f"(generated in {time.time() - t0:.1f} s)", file=sys.stderr, flush=True)
    rp = torch.from_numpy(db.row_ptr.astype(np.uint64)).to(dev)
    ci = torch.from_numpy(db.col_idx.astype(np.uint32)).to(dev)
    stream = torch.cuda.current_stream()
    # timed steps record events only around the support-counting kernels; the
    # bookkeeping launches are timed in separate steps after the timed region
    flags = (0 if args.no_timing else bm.FLAG_TIMING | bm.FLAG_TIMING_MAIN) | extra_flags
    if args.levelsync:
        flags |= bm.FLAG_LEVELSYNC
    if args.shuffle:
        flags |= bm.FLAG_SHUFFLE
    flags |= {"default": 0, "int8": bm.FLAG_INT8_MFMA, "fp4": bm.FLAG_FP4_MFMA}[args.mfma]
    dmw = args.dfs_max_words if dfs_max_words is None else dfs_max_words
    opts = _single_opts(bm, args, flags, dfs_max_words=dmw)
    model = None
    if sched == "learned":
        h = bm.bm_build(rp, ci, db.n, db.m, stream=stream)
        topts = bm.options(flags=bm.FLAG_TRACE, dfs_max_words=dmw)
        f, y = bm.bm_mine_ex(h, db.minsup, topts, stream=stream).trace()
        model = bm.Model(seed=1)
        loss = model.train(f, y, epochs=30, lr=3e-3, batch=256, stream=stream)
        print(f"# cost model trained on {len(y)} traced tasks, loss {loss:.4f}", file=sys.stderr,
              flush=True)
        del h

    def mine(h, o):
        if model is not None:
            return bm.bm_mine_batch([h], [db.minsup], model=model, opts=o, stream=stream)[0]
        return bm.bm_mine_ex(h, db.minsup, o, stream=stream)

    flush = torch.empty(2 << 30, dtype=torch.uint8, device=dev) if args.cold else None

    def step():
        h = bm.bm_build(rp, ci, db.n, db.m, stream=stream)
        if flush is not None:  # profiling runs: a cache-cold mine call
            flush.fill_(7)
        return h, mine(h, opts)

    for i in range(warmup):
        h, r = step()
        if not quiet:
            print(f"# warmup {i}: {r.stats()['wall_ms']:.2f} ms mine", file=sys.stderr, flush=True)
        del h, r
    torch.cuda.synchronize()
    stats = []
    times = []
    results = []
    t_start = time.perf_counter()
    kept = []
    for i in range(steps):
        t1 = time.perf_counter()
        h, r = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        kept.append(r)
        del h, r
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    ms_per_step = 1e3 * total / steps
    for i, r in enumerate(kept):
        stats.append(r.stats())
        results.append(r.info())
        if not quiet:
            print(f"# step {i}: {times[i] * 1e3:.2f} ms", file=sys.stderr, flush=True)
    del kept
    st = stats[-1]
    cands = st["candidates_total"]
    assert all(x == results[0] for x in results), "result changed between steps"

    # dominant kernel by total event time
    kernels, kms = _kernel_table(stats, steps)
    roofline = (_roofline(kernels, kms, st["mfma_form"]) if (not args.no_timing and kernels)
                else None)
    cold = None
    if not args.no_timing:
        # every launch kind, events around all of them, outside the timed region
        full = []
        fopts = _single_opts(bm, args, flags & ~bm.FLAG_TIMING_MAIN, dfs_max_words=dmw)
        for _ in range(3):
            h = bm.bm_build(rp, ci, db.n, db.m, stream=stream)
            full.append(mine(h, fopts).stats())
            del h
        fk, _ = _kernel_table(full, len(full))
        for k, v in fk.items():
            if k not in kernels:
                kernels[k] = dict(v, timed="separate steps with every launch timed")
        if cold_steps:
            # cache-cold mining: a 2 GiB scratch write on the same stream between
            # build and mine leaves none of the matrix in L2 or the Infinity Cache
            # (256 MB); a fill kernel, not a memset
            scratch = torch.empty(2 << 30, dtype=torch.uint8, device=dev)
            cst = []
            for i in range(cold_steps):
                h = bm.bm_build(rp, ci, db.n, db.m, stream=stream)
                scratch.fill_(i + 1)
                cst.append(mine(h, opts).stats())
                del h
            torch.cuda.synchronize()
            del scratch
            ck, _ = _kernel_table(cst, len(cst))
            cold = {"protocol": "2 GiB scratch fill between build and mine, "
                                f"{cold_steps} steps, events around the support-counting kernels",
                    "mine_ms": round(sum(s["wall_ms"] for s in cst) / len(cst), 3)}
            for k, v in ck.items():
                e = {"avg_launch_ms": v["avg_launch_ms"]}
                if "achieved_GBs" in v:
                    e["achieved_GBs"] = v["achieved_GBs"]
                    e["frac_of_hbm"] = round(v["achieved_GBs"] / HBM_PEAK_GBS, 4)
                if "achieved_TOPs" in v:
                    e["achieved_TOPs"] = v["achieved_TOPs"]
                    e["frac_of_mfma"] = round(v["achieved_TOPs"] / MFMA_PEAK_TOPS[st["mfma_form"]],
                                              4)
                cold[k] = e

    pairs = int(st["candidates"].get(2, 0))
    out = {
        "metric": "candidate supports counted/s + mine wall time at minsup; % of HBM peak",
        "value": round(cands / (ms_per_step * 1e-3), 1),
        "unit": "candidate supports/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[st["mfma_form"]],
        "data": "synthetic (seeded generator, see DESIGN.md)",
        "config": {"workload": WORKLOADS[workload], "n_tx": db.n, "n_items": db.m,
                   "minsup": db.minsup, "frequent_itemsets": st["frequent_total"],
                   "candidates": cands, "pair_candidates": pairs,
                   "longer_candidates": cands - pairs,
                   "pair_supports_per_s": round(pairs / (ms_per_step * 1e-3), 1),
                   "longer_supports_per_s": round((cands - pairs) / (ms_per_step * 1e-3), 1),
                   "frequent_items": st["n_frequent_items"],
                   "mine_ms": round(sum(s["wall_ms"] for s in stats) / len(stats), 3),
                   "dfs_tasks": st["dfs_tasks"], "host_syncs": st["host_syncs"],
                   "mode": ("levelsync" if args.levelsync or not st["dfs_tasks"] else "subtrees") +
                           ("+learned" if model is not None else "") +
                           (f"+shuffle{args.shuffle}" if args.shuffle else ""),
                   "kernels": kernels},
        "roofline": roofline,
    }
    if cold is not None:
        out["config"]["cache_cold"] = cold
    out["_db"] = db
    return out


def table_sweep(bm, torch, reps: int = 5) -> dict:
    """The paper's Table 1/2 measurements on its kind of data: a basket stand-in
    for Groceries (169 items, Zipf item popularity), mined at thresholds 1-5% on
    the first n = 2,000 .. 10,000 transactions.  Per point: build + mine wall
    time on the GPU (median of `reps`), frequent itemsets found, peak device
    memory the library held (its allocations routed through a counting
    allocator), the bitset matrix size, the mean support of the frequent
    itemsets (Table 2's measure), the C++ oracle's time, and whether the GPU
    result equals the oracle's.  Context only: the data, the subsets and the
    machine all differ from the paper's."""
    import gc
    import gen
    from oracle import cpp as ocpp
    full = gen.make_config(1)
    stream = torch.cuda.current_stream()
    live, peak = {}, [0, 0]

    def alloc(size, _s):
        t = torch.empty(size, dtype=torch.uint8, device="cuda")
        live[t.data_ptr()] = t
        peak[0] += size
        peak[1] = max(peak[1], peak[0])
        return t.data_ptr()

    def free(ptr, _s):
        t = live.pop(ptr, None)
        if t is not None:
            peak[0] -= t.numel()

    gc.collect()
    try:
        bm.bm_set_allocator(alloc, free)
        counted = True
    except bm.BmError:
        counted = False  # a handle is still alive: no memory figures
    points = []
    try:
        for n in (2000, 4000, 6000, 8000, 10000):
            rp = full.row_ptr[:n + 1].copy()
            ci = full.col_idx[:int(rp[-1])].copy()
            o = ocpp.OracleDb(rp, ci, n, full.m)
            for pct in (1, 2, 3, 4, 5):
                minsup = gen.minsup_from_ppm(pct * 10_000, n)
                t0 = time.perf_counter()
                want = o.mine_arrays(minsup)
                oracle_ms = 1e3 * (time.perf_counter() - t0)
                times = []
                for _ in range(reps):
                    peak[1] = peak[0]
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    h = bm.bm_build(rp, ci, n, full.m, stream=stream)
                    r = bm.bm_mine(h, minsup, stream=stream)
                    got = r.arrays()
                    times.append(1e3 * (time.perf_counter() - t1))
                    matrix_b = h.info()[2] * full.m * 8  # padded words x items
                    del h, r
                same = all(np.array_equal(a.astype(np.int64), b.astype(np.int64))
                           for a, b in zip(got, want[:3]))
                supp = got[2].astype(np.float64)
                points.append({
                    "threshold_pct": pct, "n": n, "minsup": minsup,
                    "gpu_build_mine_ms": round(float(np.median(times)), 3),
                    "frequent_itemsets": int(len(supp)),
                    "peak_device_mb": round(peak[1] / 2**20, 3) if counted else None,
                    "matrix_mb": round(matrix_b / 2**20, 3) if matrix_b else None,
                    "avg_support_pct": round(100.0 * float(supp.mean()) / n, 3) if len(supp) else None,
                    "oracle_ms": round(oracle_ms, 3), "equals_oracle": bool(same),
                    "table1_row": pct * 2000 == n})
    finally:
        gc.collect()
        if counted:
            bm.bm_set_allocator(None, None)
    paper = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")))
    return {"data": "basket stand-in (10,000 x 169, Zipf 1.1), first n rows; thresholds as "
                    "minsup = ceil(pct * n / 100), frequent iff supp >= minsup",
            "points": points, "paper": {"table1": paper["table1"], "table2": paper["table2"],
                                        "hardware": "not stated"}}


def blocked_run(bm, torch, workload: int = 3, block_rows: int = 250_000, reps: int = 2) -> dict:
    """Out-of-core mining of a workload from its host CSR, block_rows transactions
    on the device at a time (every level re-reads the CSR over the host link),
    against in-core build + mine from the same host CSR."""
    import gen
    db = gen.make_config(workload)
    t_blk, t_in = [], []
    res = None
    for _ in range(reps + 1):  # the first call warms the pool
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = bm.bm_mine_blocked(db.row_ptr, db.col_idx, db.n, db.m, db.minsup, block_rows)
        torch.cuda.synchronize()
        t_blk.append(1e3 * (time.perf_counter() - t0))
        res = r.info()
        t0 = time.perf_counter()
        h = bm.bm_build(db.row_ptr, db.col_idx, db.n, db.m)
        r2 = bm.bm_mine(h, db.minsup)
        torch.cuda.synchronize()
        t_in.append(1e3 * (time.perf_counter() - t0))
        assert r2.info() == res
        del h, r, r2
    return {"workload": WORKLOADS[workload], "block_rows": block_rows,
            "blocks": -(-db.n // block_rows), "frequent_itemsets": res[0],
            "blocked_ms": round(float(np.median(t_blk[1:])), 3),
            "in_core_build_mine_ms": round(float(np.median(t_in[1:])), 3),
            "note": "both from host CSR (upload included); the blocked run re-reads the CSR "
                    "over the host link once per level"}


def _secondary(args, bm, torch, dev):
    """Shorter runs of the batched and the T40-style workloads, for the record."""
    global WORKLOAD
    sec = {}
    WORKLOAD = 4
    b = run_batched(args, bm, torch, dev, steps=10, warmup=3)
    sec["batch_256"] = {"ms_per_step_by_mode": {k: v["ms_per_step"]
                                                for k, v in b["config"]["modes"].items()},
                        "mine_ms_by_mode": {k: v["mine_ms"] for k, v in b["config"]["modes"].items()},
                        "candidates": b["config"]["candidates"],
                        "value_learned": b["value"], "roofline": b["roofline"]}
    t40 = {}
    WORKLOAD = 5  # the T40-style workload's traffic records
    for name, kw in (("default", {}),
                     ("depth_first_plain", {"extra_flags": bm.FLAG_DEPTH_FIRST,
                                            "dfs_max_words": 0xFFFFFFFF}),
                     ("depth_first_learned", {"extra_flags": bm.FLAG_DEPTH_FIRST,
                                              "dfs_max_words": 0xFFFFFFFF, "sched": "learned"})):
        r = run_single(args, bm, torch, dev, 5, 10, 3, cold_steps=3 if name == "default" else 0,
                       quiet=True, **kw)
        e = {"ms_per_step": r["ms_per_step"], "mine_ms": r["config"]["mine_ms"],
             "candidates": r["config"]["candidates"], "value": r["value"]}
        if name == "default":
            e["roofline"] = r["roofline"]
            e["cache_cold"] = r["config"].get("cache_cold")
            e["pair_candidates"] = r["config"]["pair_candidates"]
            e["longer_candidates"] = r["config"]["longer_candidates"]
        t40[name] = e
        print(f"# T40 {name}: {r['ms_per_step']} ms/step", file=sys.stderr, flush=True)
    sec["quest_t40_1M"] = t40
    WORKLOAD = None
    return sec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", type=int, default=3, choices=sorted(WORKLOADS),
                    help="1-3, 5: one database; 4: the batch of 256 (mode comparison)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the shorter batched and T40-style runs after the headline")
    ap.add_argument("--cold", action="store_true",
                    help="profiling: write 2 GiB between build and mine in every step (the fill "
                         "is inside the timed step)")
    ap.add_argument("--sweep", action="store_true",
                    help="only the Table 1/2-style sweep (threshold x transactions) as JSON")
    ap.add_argument("--no-timing", action="store_true", help="do not record per-kernel events")
    ap.add_argument("--mfma-min-children", type=int, default=0)
    ap.add_argument("--split-words", type=int, default=0)
    ap.add_argument("--mfma", choices=["default", "int8", "fp4"], default="default",
                    help="form of the Gram kernels' MFMA")
    ap.add_argument("--mfma-big-children", type=int, default=0)
    ap.add_argument("--levelsync", action="store_true",
                    help="plain level-synchronous miner (no depth-first phase)")
    ap.add_argument("--dfs-threads", type=int, default=0)
    ap.add_argument("--dfs-max-words", type=int, default=0)
    ap.add_argument("--shuffle", type=int, default=0, help="random subtree-task order with this seed")
    ap.add_argument("--sched", choices=["none", "learned"], default="none",
                    help="learned: order subtree tasks by a cost model trained on a traced run")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="instead of mining, copy a buffer of this size (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the library runs on one GPU "
              "and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

    if args.copy_probe_mb:
        n = args.copy_probe_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4}), flush=True)
        return

    import paper_2412_19420_amd as bm

    if args.sweep:
        print(json.dumps(table_sweep(bm, torch)), flush=True)
        return

    global WORKLOAD
    WORKLOAD = args.workload
    if args.workload == 4:
        print(json.dumps(run_batched(args, bm, torch, dev)), flush=True)
        return

    out = run_single(args, bm, torch, dev, args.workload, args.steps, args.warmup, sched=args.sched)
    db = out.pop("_db")
    if not args.no_secondary and args.workload == 3:
        out["config"]["secondary"] = _secondary(args, bm, torch, dev)
        out["config"]["secondary"]["table_sweep"] = table_sweep(bm, torch)
        out["config"]["secondary"]["out_of_core"] = blocked_run(bm, torch)
        WORKLOAD = args.workload
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(db)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
