"""Benchmark of the predicate-transfer phase on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload star]

A step is one whole transfer phase (local predicates, forward pass, backward
pass: every kernel of the path) over the star schema: a 100 M-row fact table
with four int32 foreign keys into dimensions of 2 M, 200 k, 10 k and 25 rows,
range predicates keeping 1 % and 20 % of the first two, Bloom filters with
512-bit blocks, k = 3 and 10 bits per key. Inputs are synthetic, seeded and
already resident in HBM when timing starts.

Prints one JSON line: rows probed per second (the rows every probe step
scans, summed over both passes), the fact-table probe kernel against the HBM
roofline, and the CPU oracle timed on the host beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published peak


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="star", choices=["star", "chain", "snowflake", "batch", "served"])
    ap.add_argument("--queries", type=int, default=2000, help="served: queries per load level")
    ap.add_argument("--loads", default="0.5,0.9,1.5",
                    help="served: offered loads (arrival rate x mean solo latency)")
    ap.add_argument("--no-tune", action="store_true",
                    help="batch: B = 512, k = 3, 10 bits per key for every problem instead of autotuning")
    ap.add_argument("--problems", type=int, default=256, help="batch: number of problems")
    ap.add_argument("--bpk", type=int, default=None, help="bits per key (default 10; snowflake 12)")
    ap.add_argument("--no-append", action="store_true",
                    help="builds rescan the table instead of reading keys appended by its probe")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-join", action="store_true", help="star: skip the join-phase and exact-filter timings")
    ap.add_argument("--no-prune", action="store_true", help="star, snowflake: skip the transfer-path-pruning timing")
    ap.add_argument("--hold", type=float, default=0.0,
                    help="served: hold a lone query beside a running batch for up to this many mean solo "
                         "service times, for another query to batch with")
    ap.add_argument("--check", action="store_true", help="compare the result with the oracle")
    ap.add_argument("--no-kernel-events", action="store_true",
                    help="time the steps without the per-kernel HIP events (no roofline figure)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after timing, copy 1 GiB device to device three times (a kernel of known "
                         "traffic to scale hardware byte counters by)")
    return ap.parse_args()


# Sources the probe kernels are compiled from: counters taken on other
# sources do not describe the kernel that runs.
PROBE_SOURCES = ["include/pt.h", "paper_2307_15255_amd/csrc/pt_internal.hpp",
                 "paper_2307_15255_amd/csrc/pt_common.hpp", "paper_2307_15255_amd/csrc/probe_impl.hpp",
                 "paper_2307_15255_amd/csrc/k_probe_512.hip", "paper_2307_15255_amd/csrc/k_probe_gen.hip"]


def probe_source_hash() -> str:
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for rel in PROBE_SOURCES:
        with open(os.path.join(here, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str, dom_key) -> tuple[float | None, str | None]:
    """HBM bytes per launch of the dominant kernel as two rocprofv3 --pmc
    runs measured them (FETCH_SIZE, WRITE_SIZE, scaled by a copy kernel of
    known traffic), from the committed summary under profiles/, and that
    file's name; (None, None) unless the counters were taken on the probe
    sources that are built now."""
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", f"probe_{workload}_fact_traffic.json")
    if dom_key[0] != "probe" or dom_key[2] != 1 or not os.path.exists(path):
        return None, None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != probe_source_hash() or rec.get("table") != dom_key[1]:
        return None, None
    return float(rec["traffic_bytes"]), os.path.relpath(path, here)


def host_cpu() -> str:
    """Logical CPUs of the host and its model name."""
    model = "unknown model"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{host_cores()} logical CPUs available ({os.cpu_count()} online), {model}"


def host_cores() -> int:
    """Logical CPUs this process may run on, at most 16 (the share of the
    host one GPU comes with)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


def rows_probed(prob, order_src_dst) -> int:
    """Rows scanned by probe steps: every table with at least one incoming
    edge in a pass is scanned once in that pass."""
    src, dst = order_src_dst
    fwd = {d for d in dst}
    bwd = {s for s in src}
    return sum(prob.n_rows(t) for t in fwd) + sum(prob.n_rows(t) for t in bwd)


def orientation(prob):
    src, dst = [], []
    for e, (u, _, v, _) in enumerate(prob.edges):
        if prob.orient is not None:
            first = prob.orient[e] > 0
        else:
            nu, nv = prob.n_rows(u), prob.n_rows(v)
            first = nu < nv or (nu == nv and u < v)
        src.append(u if first else v)
        dst.append(v if first else u)
    return src, dst


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the transfer path is built and timed on a single MI355X; "
              "the library has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2307_15255_amd import pt
    from paper_2307_15255_amd import workloads as W

    if args.workload == "batch":
        return bench_batch(args, torch, pt, W)
    if args.workload == "served":
        return bench_served(args, torch, pt, W)

    t0 = time.time()
    if args.workload == "star":
        prob = W.star(seed=args.seed)
        cfg = {"workload": "star", "fact_rows": 100_000_000, "dims": list(W.STAR_DIMS),
               "fk_dtype": "int32", "predicates": "D0 1%, D1 20%", "block_bits": 512, "k": 3,
               "bits_per_key": 10}
    elif args.workload == "snowflake":
        prob = W.snowflake(seed=args.seed)
        cfg = {"workload": "snowflake", "rows": W.SNOWFLAKE_ROWS, "key_dtype": "int64",
               "fk_distribution": "Zipf(1.1)", "cycle": "F-D2-D3", "block_bits": 512, "k": 3,
               "bits_per_key": args.bpk or 12}
    else:
        prob = W.chain(seed=args.seed)
        cfg = {"workload": "chain", "rows": [1000, 10000, 1000], "block_bits": 512, "k": 3,
               "bits_per_key": 10}
    bpk = cfg["bits_per_key"] = args.bpk or cfg["bits_per_key"]
    gen_s = time.time() - t0
    dp = pt.DeviceProblem(prob)
    tr = pt.Transfer(dp, pt.params(512, 3, bpk, pt.PT_FLAG_NO_APPEND if args.no_append else 0))
    torch.cuda.synchronize()
    print(f"# inputs ready in {time.time() - t0:.1f}s (generation {gen_s:.1f}s)", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        tr.run()
    torch.cuda.synchronize()

    # One more untimed step with HIP events around every launch (on the
    # stream each is launched on) names the dominant launch, the (step,
    # table, pass) with the largest time, and gives the per-kernel breakdown.
    dom_key, breakdown = None, {}
    if not args.no_kernel_events:
        pt.pt_profile_enable(1)
        tr.run()
        torch.cuda.synchronize()
        pt.pt_profile_enable(False)
        by_key: dict[tuple, list] = {}
        for r in pt.pt_profile_read(1 << 16):
            by_key.setdefault((r["name"], r["table"], r["pass_"]), []).append(r["ms"])
        if by_key:
            dom_key = max(by_key, key=lambda k: sum(by_key[k]))
            breakdown = {f"{k[0]}:t{k[1]}:p{k[2]}": round(float(sum(v)), 4)
                         for k, v in sorted(by_key.items(), key=lambda kv: -sum(kv[1]))[:8]}

    # the timed steps record events around the dominant launch only, so the
    # other launches run back to back as they do without profiling
    if dom_key is not None:
        pt.pt_profile_only(*dom_key)
        pt.pt_profile_enable(1)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        tr.run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    pt.pt_profile_enable(False)
    pt.pt_profile_only(None)
    records = pt.pt_profile_read(1 << 16)

    ms_per_step = elapsed * 1000 / args.steps
    n_probed = rows_probed(prob, orientation(prob))
    value = n_probed / (ms_per_step / 1000) / 1e9

    if args.calibrate_copy:
        # an elementwise kernel of known traffic: reads 1 GiB, writes 1 GiB
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    if not records:
        print(json.dumps({"metric": "G rows probed/s", "value": round(value, 3), "unit": "G rows/s",
                          "ms_per_step": round(ms_per_step, 4), "steps": args.steps,
                          "note": "no per-kernel events"}), flush=True)
        return
    # the dominant kernel's average over the timed steps
    dom = [r for r in records if (r["name"], r["table"], r["pass_"]) == dom_key]
    dom_ms = float(np.mean([x["ms"] for x in dom]))
    dom_bytes = dom[0]["bytes"]
    achieved = dom_bytes / (dom_ms / 1000) / 1e9

    out = {
        "metric": "G rows probed/s",
        "value": round(value, 3),
        "unit": "G rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64" if args.workload == "snowflake" else "int32",
        "data": "synthetic",
        "config": cfg,
        "rows_probed_per_step": n_probed,
        "roofline": {
            "bound": "hbm",
            "kernel": f"{dom_key[0]} table {dom_key[1]} pass {dom_key[2]}",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "algorithmic_bytes": dom_bytes,
            "avg_ms": round(dom_ms, 5),
        },
        "kernel_ms": breakdown,
        "kernel_ms_from": "one untimed step with events on every launch",
    }

    if args.workload == "star" and not args.no_join:
        out["join"] = bench_join(args, torch, pt, prob, dp, tr)
        out["exact_filters"] = bench_exact(args, torch, pt, prob, dp, tr, ms_per_step)
    if args.workload in ("star", "snowflake") and not args.no_prune:
        out["pruned"] = bench_prune(args, torch, pt, prob, dp, tr, bpk, ms_per_step)

    if args.calibrate_copy:
        out["calibration_copy_bytes"] = 1 << 30
    traffic, source = measured_traffic(args.workload, dom_key)
    out["roofline"]["traffic"] = traffic
    if source:
        out["roofline"]["traffic_source"] = source

    if args.check or not args.no_cpu_baseline:
        import oracle

        def median_run(threads):
            # the whole workload, repeated until about 8 s of oracle work (at
            # least once); the median run and the last result
            runs = []
            while not runs or (sum(runs) < 8 and len(runs) < 5):
                t = time.perf_counter()
                res = oracle.transfer(prob, 512, 3, bpk, threads=threads)
                runs.append(time.perf_counter() - t)
            return float(np.median(runs)), len(runs), res

        cpu_s, n_runs, ref = median_run(1)
        if not args.no_cpu_baseline:
            # the oracle's row split over every available core (whole bitmap
            # words per thread, private filter copies OR-ed): bit-exact with
            # the one-thread run, checked here
            cores = host_cores()
            all_s, all_runs, ref_all = median_run(cores)
            same = all(np.array_equal(a, b) for a, b in zip(ref.bitmaps, ref_all.bitmaps))
            out["cpu_baseline"] = {
                "value": round(n_probed / all_s / 1e9, 4),
                "unit": "G rows/s",
                "cores": cores,
                "kind": "oracle",
                "sample": f"the whole workload ({n_probed} rows probed), median of {all_runs} runs of "
                          f"{all_s:.2f} s on {cores} threads; host: {host_cpu()}",
                "bit_exact_with_single_thread": bool(same),
                "single_thread": {"value": round(n_probed / cpu_s / 1e9, 4), "cores": 1,
                                  "sample": f"median of {n_runs} runs of {cpu_s:.2f} s"},
            }
        if args.check:
            ok = all(np.array_equal(tr.bitmap(t), ref.bitmaps[t]) for t in range(prob.n_tables))
            out["check"] = "bit-exact" if ok else "MISMATCH"
    print(json.dumps(out), flush=True)


def bench_join(args, torch, pt, prob, dp, tr) -> dict:
    """The join phase (Sec. 3.3) on the star, from the fact table, timed
    with HIP events apart from the transfer steps: on the tables the
    transfer phase reduced, and on the tables reduced by their local
    predicates only (the plan without predicate transfer), which hands the
    join every fact row."""
    local = []
    for t in range(prob.n_tables):
        bm = torch.empty(pt.bitmap_words(prob.n_rows(t)), dtype=torch.int64, device="cuda")
        cols = list(dp.columns[t].values())
        preds = [(prob.col_index(t, c), op, lo, hi) for tt, c, op, lo, hi in prob.preds if tt == t]
        pt.pt_local_filter(cols, preds, prob.n_rows(t), bm)
        local.append(bm)
    j = pt.Join(dp, root=0, out_cap=1 << 22)
    res = {}
    for name, bitmaps in (("after_transfer", tr.bitmaps), ("after_local_filters_only", local)):
        for _ in range(2):
            j.run(bitmaps)
        j.check_status()
        times = []
        for _ in range(max(3, min(args.steps, 20))):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            j.run(bitmaps)
            b.record()
            b.synchronize()
            times.append(a.elapsed_time(b))
        j.check_status()
        res[name] = {"ms": round(float(np.median(times)), 4), "tuples": int(j.n_out.item())}
    res["tuples_equal"] = res["after_transfer"]["tuples"] == res["after_local_filters_only"]["tuples"]
    res["root"] = "fact table; dimensions added in edge order as hash-table build sides"
    return res


def bench_exact(args, torch, pt, prob, dp, tr, bloom_ms: float) -> dict:
    """The same transfer with exact filters (PT_FLAG_EXACT: key sets, every
    transfer a semi-join, Sec. 3.2), timed apart from the Bloom steps: its
    time per step against the Bloom step, and the rows each leaves."""
    ex = pt.Transfer(dp, pt.params(512, 3, 10, pt.PT_FLAG_EXACT))
    for _ in range(2):
        ex.run()
    ex.check_status()
    times = []
    for _ in range(max(3, min(args.steps, 20))):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        ex.run()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    ms = float(np.median(times))
    res = {"ms_per_step": round(ms, 4), "vs_bloom_step": round(ms / bloom_ms, 2),
           "rows_left": [int(x) for x in ex.counts.cpu().tolist()],
           "rows_left_bloom": [int(x) for x in tr.counts.cpu().tolist()],
           "workspace_GB": round(ex.ws_bytes / 2**30, 2)}
    del ex
    torch.cuda.empty_cache()
    return res


def bench_prune(args, torch, pt, prob, dp, tr, bpk: int, full_ms: float) -> dict:
    """The same transfer with transfer path pruning (PT_FLAG_PRUNE, Sec. 3.2:
    a table that still holds every row sends no filter), timed apart from
    the full steps: its time per step against the full step, and whether it
    left the same rows (it does when every foreign key references an
    existing key, as in these workloads)."""
    pr = pt.Transfer(dp, pt.params(512, 3, bpk, pt.PT_FLAG_PRUNE))
    for _ in range(2):
        pr.run()
    pr.check_status()
    times = []
    for _ in range(max(3, min(args.steps, 20))):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        pr.run()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    ms = float(np.median(times))
    same = all(torch.equal(x, y) for x, y in zip(pr.bitmaps, tr.bitmaps))
    res = {"ms_per_step": round(ms, 4), "vs_full_step": round(ms / full_ms, 3),
           "rows_left": [int(x) for x in pr.counts.cpu().tolist()], "bits_equal_full": bool(same)}
    del pr
    torch.cuda.empty_cache()
    return res


def bench_batch(args, torch, pt, W):
    """256 independent chain and star problems (tables log-uniform on
    [10 k, 5 M] rows) run as one batch: one persistent launch per step (a
    captured graph). Beside it, the same problems one at a time with plain
    pt_transfer launches."""
    from paper_2307_15255_amd import autotune
    t0 = time.time()
    probs = W.batch(seed=args.seed, n_problems=args.problems)
    dps = [pt.DeviceProblem(p) for p in probs]
    torch.cuda.synchronize()
    print(f"# batch inputs ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    tiles = None
    if args.no_tune:
        ps, tune_s = [pt.params(512, 3, 10) for _ in probs], 0.0
    else:
        t1 = time.time()
        ps, _ = autotune.tune(probs)
        ps, tiles = autotune.tune_tiles(dps, ps)
        tune_s = time.time() - t1
    chosen: dict[str, int] = {}
    for p in ps:
        key = f"B{p.block_bits}/k{p.k}/bpk{p.bits_per_key}"
        chosen[key] = chosen.get(key, 0) + 1
    bt = pt.Batch(dps, ps)
    n_launch, n_probed = bt.info()
    for _ in range(args.warmup):
        bt.run()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        bt.run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1000 / args.steps
    # the persistent batch kernel timed with HIP events on its stream (eager
    # runs: the counter reset, then the kernel between the events)
    pt.pt_profile_enable(1)
    for _ in range(3):
        bt.run(eager=True)
    torch.cuda.synchronize()
    pt.pt_profile_enable(False)
    recs = [r for r in pt.pt_profile_read(4096) if r["name"] == "batch"]
    dom_ms = float(np.mean([r["ms"] for r in recs]))
    dom = dict(recs[0], ms=dom_ms)
    achieved = dom["bytes"] / (dom["ms"] / 1000) / 1e9
    # one query at a time, plain launches
    trs = [pt.Transfer(dp, p) for dp, p in zip(dps, ps)]
    for tr in trs:
        tr.run()
    torch.cuda.synchronize()
    reps = max(1, min(5, args.steps // 10))
    t = time.perf_counter()
    for _ in range(reps):
        for tr in trs:
            tr.run()
    torch.cuda.synchronize()
    single_ms = (time.perf_counter() - t) * 1000 / reps
    out = {
        "metric": "G rows probed/s",
        "value": round(n_probed / (ms / 1000) / 1e9, 3),
        "unit": "G rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "batch", "problems": len(probs), "rows": sum(sum(d.n_rows) for d in dps),
                   "table_rows": "log-uniform [10k, 5M]", "params": chosen, "autotune_s": round(tune_s, 2),
                   "tile_rows": ps[0].tile_rows,
                   "tile_search_ms": tiles["measured_ms"] if tiles else None,
                   "launches_per_run": n_launch},
        "rows_probed_per_step": n_probed,
        "one_at_a_time": {"ms_per_step": round(single_ms, 4),
                          "value": round(n_probed / (single_ms / 1000) / 1e9, 3),
                          "speedup_of_batch": round(single_ms / ms, 2)},
        "roofline": {"bound": "hbm", "kernel": f"k_batch (one persistent launch, {dom['table']} tasks)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "algorithmic_bytes": dom["bytes"], "avg_ms": round(dom["ms"], 5),
                     "bytes_counted": "key columns and bitmaps of every probe and local filter"},
    }
    if not args.no_cpu_baseline:
        import oracle
        # a bounded sample: the first problems until about 8 s of oracle
        # work, on every available core (the oracle's row split), then the
        # same problems on one thread
        cores = host_cores()
        t = time.perf_counter()
        rows = 0
        for i, prob in enumerate(probs):
            p = ps[i]
            oracle.transfer(prob, p.block_bits, p.k, p.bits_per_key, threads=cores)
            rows += rows_probed(prob, orientation(prob))
            if time.perf_counter() - t > 8:
                break
        cpu_s = time.perf_counter() - t
        t = time.perf_counter()
        for prob, p in zip(probs[:i + 1], ps):
            oracle.transfer(prob, p.block_bits, p.k, p.bits_per_key)
        one_s = time.perf_counter() - t
        out["cpu_baseline"] = {"value": round(rows / cpu_s / 1e9, 4), "unit": "G rows/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"the first {i + 1} problems ({rows} rows probed in {cpu_s:.2f} s on "
                                         f"{cores} threads); host: {host_cpu()}",
                               "single_thread": {"value": round(rows / one_s / 1e9, 4), "cores": 1,
                                                 "sample": f"the same problems in {one_s:.2f} s"}}
    print(json.dumps(out), flush=True)


def bench_served(args, torch, pt, W):
    """The star schema resident in HBM (plus int64 twins of two key pairs);
    a Poisson stream of random 2-5-table queries at offered loads rho =
    arrival rate x mean solo latency; the batching server against one query
    at a time with plain pt_transfer launches, same arrivals."""
    from paper_2307_15255_amd import serve as S
    t0 = time.time()
    res = S.ResidentStar(seed=args.seed)
    torch.cuda.synchronize()
    print(f"# resident tables ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    rng = np.random.default_rng(args.seed)
    arena = 8 << 30
    # every query of the run, drawn up front; the single-query arena fits the largest
    loads = [float(x) for x in args.loads.split(",")]
    warm = [S.random_query(rng, -1 - i) for i in range(48)]
    sample = [S.random_query(rng, -100 - i) for i in range(64)]
    streams = [[S.random_query(rng, i) for i in range(args.queries)] for _ in loads]
    sizer = S.GpuExecutor(res, slots=0)
    single = max(sizer.single_need(q) for q in warm + sample + [q for qs in streams for q in qs])
    del sizer
    ex = S.GpuExecutor(res, slots=2, arena_bytes=arena, single_arena_bytes=single)
    for q in warm + sample + [q for qs in streams for q in qs]:  # descriptors built before any clock starts
        ex.device_problem(q)
    print(f"# executor ready (single-query workspace {single / 2**30:.2f} GiB)", file=sys.stderr, flush=True)
    # solo latency: a sample of queries, each run alone after a warm-up
    S.one_at_a_time(warm, ex)
    S.serve(warm, ex, budget_bytes=2 * arena, slots=2, max_batch=64, batch_bytes=arena)
    solo = S.one_at_a_time(sample, ex)
    lat = np.array(sorted(solo.service.values()))
    s1 = float(lat.mean())  # mean service time of a query run alone
    slow = sorted(sample, key=lambda q: -solo.service[q.qid])[:3]
    print(f"# solo service time mean {s1 * 1e3:.3f} ms, median {np.median(lat) * 1e3:.3f}, "
          f"max {lat[-1] * 1e3:.3f}; slowest: "
          f"{[(q.dims, q.wide, q.preds, round(solo.service[q.qid] * 1e3, 2)) for q in slow]}",
          file=sys.stderr, flush=True)
    levels = []
    for rho, qs in zip(loads, streams):
        for q, t in zip(qs, S.poisson_arrivals(rng, len(qs), rho / s1)):
            q.arrival = float(t)
        srv = S.serve(qs, ex, budget_bytes=2 * arena, slots=2, max_batch=64, batch_bytes=arena,
                      hold=args.hold * s1)
        torch.cuda.synchronize()
        print(f"# load {rho}: served in {srv.wall:.2f} s", file=sys.stderr, flush=True)
        fifo = S.one_at_a_time(qs, ex)
        torch.cuda.synchronize()
        rows = 0
        for q in qs:
            prob, _ = res.problem(q)
            rows += rows_probed(prob, orientation(prob))
        levels.append({
            "rho": rho, "qps": round(rho / s1, 1), "queries": len(qs),
            "served": {"p50_ms": round(srv.percentile(50) * 1e3, 3), "p99_ms": round(srv.percentile(99) * 1e3, 3),
                       "G_rows_probed_per_s": round(rows / srv.wall / 1e9, 3), "batches": len(srv.batches),
                       "mean_batch": round(len(qs) / len(srv.batches), 2),
                       "rejected": len(srv.rejected), "timed_out": len(srv.timed_out),
                       "host_launch_ms_per_batch": round(srv.launch_host_s * 1e3 / max(1, len(srv.batches)), 3),
                       "peak_admitted_GB": round(srv.peak_bytes / 2**30, 2)},
            "one_at_a_time": {"p50_ms": round(fifo.percentile(50) * 1e3, 3),
                              "p99_ms": round(fifo.percentile(99) * 1e3, 3),
                              "G_rows_probed_per_s": round(rows / fifo.wall / 1e9, 3)},
        })
        print(f"# load {rho}: served p50/p99 {levels[-1]['served']['p50_ms']}/{levels[-1]['served']['p99_ms']} ms, "
              f"alone {levels[-1]['one_at_a_time']['p50_ms']}/{levels[-1]['one_at_a_time']['p99_ms']} ms",
              file=sys.stderr, flush=True)
    top = levels[-1]
    out = {
        "metric": "served p99 latency",
        "value": top["served"]["p99_ms"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.queries,
        "warmup": len(warm),
        "ms_per_step": round(top["served"]["p50_ms"], 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32+int64",
        "data": "synthetic",
        "config": {"workload": "served", "resident": "star 100M fact + dims (2M, 200k, 10k, 25), int64 twins "
                   "of (k0, D0.pk) and (k1, D1.pk)", "query": "fact + 1-4 dims, 1-2 predicates with selectivity "
                   "log-uniform [0.1%, 50%]", "arrivals": "Poisson", "solo_latency_ms": round(s1 * 1e3, 3),
                   "slots": 2, "max_batch": 64, "arena_GB_per_slot": arena / 2**30,
                   "hold_ms": round(args.hold * s1 * 1e3, 3)},
        "loads": levels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
