"""Benchmark of the fused filter -> hash join -> hash group-by pipeline on one
MI355X.

Workload (the star-schema configuration): a 600M-row fact table (int32
fk_a -> dim A of 1.5M rows, int32 fk_b -> dim B of 10k rows, int32 date
uniform over [0, 2557), int64 price x100 uniform over [100, 1e7), int8 flag
in {0, 1, 2}), filter date < 767 (about 30% of rows), inner join with both
dims, group by (dim B region over 25 values, flag), SUM/COUNT/AVG/MIN/MAX of
price. One step is one rel_pipeline call: build both dim hash tables, the
fused filter-probe-aggregate pass over the fact table, and the group
finalize. The headline keeps both dims in open-addressing hash tables
(REL_TUNE_NO_DIRECT); the same plan with the dense dim keys in direct tables
is reported beside it. Inputs are generated (seeded, synthetic) and resident
in HBM before timing starts.

Prints one JSON line: input rows/s over the whole step, the roofline of the
dominant kernel (the fused pass) from HIP events on its launch stream, the
streaming-read ceiling measured in the same run, and the single-threaded CPU
oracle timed on a bounded sample of the same rows; then the small join +
group-by as latency, batches, serving and the standalone operators.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FACT_BYTES_PER_ROW = 4 + 4 + 4 + 8 + 1  # fk_a, fk_b, date, price, flag
METRIC = "input rows/s & % HBM peak, join+groupby; batched vs per-query launch; p99 lat"
AGGS = [("sum", 3), ("count", None), ("avg", 3), ("min", 3), ("max", 3)]
TERMS = [(2, "lt", 767)]
KEYS = [("dim", 1), ("fact", 4)]


# Sources that define the fused kernel and its launch configuration; a
# traffic figure taken with rocprofv3 counters is reported only while they
# are unchanged.
KERNEL_SOURCES = ["device.h", "internal.h", "group_lds.h", "pipeline_kernel.h", "pipeline.hip", "api.cpp"]
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "pipeline_fused_hash_star600m.json")
TRAFFIC_PROFILE_DIRECT = os.path.join(ROOT, "profiles", "pipeline_fused_star600m.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2508_04701_amd", "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(n: int, path: str):
    """HBM bytes per launch of the fused kernel from the committed counter
    summary at `path` (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of
    known size), or None if it was taken on other kernel sources or another
    size."""
    try:
        with open(path) as f:
            prof = json.load(f)
    except (OSError, ValueError):
        return None
    if prof.get("kernel_sources_sha256") != kernel_sources_sha256() or prof.get("fact_rows") != n:
        return None
    return prof["fetch_bytes"] + prof["write_bytes"]


def star_run(args, torch, rel, fact, dims, t) -> dict:
    """Times the star-schema step (dim builds, fused pass, merge, finalize)
    with HIP events over args.steps launches; the fused kernel class from the
    library's per-kernel events on its launch stream."""
    plan = rel.PreparedPipeline(fact, TERMS, dims, KEYS, AGGS, max_groups=128, t=t)
    for _ in range(args.warmup):
        plan.launch()
    torch.cuda.synchronize()
    keys, aggs = plan.result()
    o = torch.argsort(keys[0].long() * 4 + keys[1].long())
    result = [keys[0][o], keys[1][o]] + [a[o] for a in aggs]
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rel.profile_read()
    rel.profile_enable(True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(args.steps):
        plan.launch()
    stop.record(stream)
    torch.cuda.synchronize()
    rel.profile_enable(False)
    prof = rel.profile_read()
    fused_ms, fused_n = prof["pipeline_fused"]
    del plan
    return {"ms_per_step": start.elapsed_time(stop) / args.steps,
            "fused_kernel_ms": fused_ms / max(1, fused_n), "groups": int(keys[0].numel()),
            "breakdown_ms_per_step": {k: round(v[0] / max(1, args.steps), 4)
                                      for k, v in prof.items() if v[1]},
            "result": result}


def stream_ceiling(args, torch, rel, cols) -> dict:
    """The streaming-read ceiling measured in the same run: rel_stream_read
    over the same columns (each byte read once, nothing else done), timed by
    the library's per-kernel events."""
    d = torch.zeros(1, dtype=torch.int64, device="cuda")
    nbytes = sum(c.numel() * c.element_size() for c in cols)
    for c in cols:
        rel.stream_read_async(c, d)
    torch.cuda.synchronize()
    rel.profile_read()
    rel.profile_enable(True)
    for _ in range(args.stream_reps):
        for c in cols:
            rel.stream_read_async(c, d)
    torch.cuda.synchronize()
    rel.profile_enable(False)
    ms, launches = rel.profile_read()["stream_read"]
    per_pass = ms / args.stream_reps
    gbs = nbytes / (per_pass * 1e-3) / 1e9
    return {"bytes": nbytes, "ms": per_pass, "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS,
            "launches_per_pass": launches // args.stream_reps,
            "workload": "rel_stream_read over the five fact columns, one launch per column"}


def bench_c1(args, torch, datagen, rel) -> dict:
    """The small join + group-by (65,536 build rows with unique int32 keys and
    a 64-value group attribute; 1,048,576 probe rows over 72,090 key values;
    SUM(value), COUNT(*) by group) as one rel_pipeline step with its build
    side in a hash table. Its 13.1 MB fit the caches, so it is reported as
    latency: warm (back-to-back steps) and cold (a 1 GiB buffer written
    before each step evicts the Infinity Cache)."""
    d = datagen.join_groupby()
    fact = [torch.from_numpy(d["probe_key"]).cuda(), torch.from_numpy(d["probe_val"]).cuda()]
    dims = [dict(fk=0, key=torch.from_numpy(d["build_key"]).cuda(),
                 payload=torch.from_numpy(d["build_grp"]).cuda())]
    aggs = [("sum", 1), ("count", None)]
    n_probe, n_build = len(d["probe_key"]), len(d["build_key"])
    alg = 12 * n_probe + 8 * n_build
    out = {"workload": f"join {n_build} build x {n_probe} probe rows (int32 keys, hash table), "
                       "group by the build side's attribute (64 groups), SUM(value), COUNT(*)",
           "algorithmic_bytes": alg}
    flush = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    for name, t in (("hash", rel.tuning(flags=rel.TUNE_NO_DIRECT)), ("direct", None)):
        plan = rel.PreparedPipeline(fact, [], dims, [("dim", 0)], aggs, 64, t)
        for _ in range(3):
            plan.launch()
        torch.cuda.synchronize()
        groups = int(plan.result()[0][0].numel())
        res = {}
        for mode in ("warm", "cold"):
            times = []
            prof = {}
            for _ in range(args.c1_reps):
                if mode == "cold":
                    flush.fill_(len(times) & 0xFF)
                start = torch.cuda.Event(enable_timing=True)
                stop = torch.cuda.Event(enable_timing=True)
                rel.profile_enable(True)
                start.record(stream)
                plan.launch()
                stop.record(stream)
                torch.cuda.synchronize()
                rel.profile_enable(False)
                for k, v in rel.profile_read().items():
                    if v[1]:
                        prof[k] = prof.get(k, 0.0) + v[0]
                times.append(start.elapsed_time(stop))
            med = float(np.median(times))
            res[mode] = {"median_ms": med, "min_ms": float(min(times)),
                         "rows_per_s": n_probe / (med * 1e-3),
                         "frac": alg / (med * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "kernel_ms": {k: round(v / args.c1_reps, 5) for k, v in prof.items()}}
        res["groups"] = groups
        out[name] = res
        del plan
    del flush
    torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(d: dict, n_fact: int, target_s: float) -> dict:
    """The oracle (single-threaded, as it stands) on the first S fact rows,
    S chosen so that it runs for about target_s seconds."""
    import oracle

    def run(s):
        fact = [d["fk_a"][:s], d["fk_b"][:s], d["date"][:s], d["price"][:s], d["flag"][:s]]
        dims = [dict(fk=0, key=d["dim_a_key"], payload=None),
                dict(fk=1, key=d["dim_b_key"], payload=d["dim_b_region"])]
        t0 = time.perf_counter()
        oracle.pipeline(fact, TERMS, dims, KEYS, AGGS)
        return time.perf_counter() - t0

    # two short runs separate the fixed cost (building the dim maps) from
    # the per-row cost, so that the sample lands near target_s
    probe = min(n_fact, 2_000_000)
    t1 = run(probe)
    t2 = run(min(n_fact, 2 * probe)) if n_fact > probe else t1
    per_row = max((t2 - t1) / probe, 1e-9) if n_fact > probe else t1 / max(probe, 1)
    fixed = max(t1 - per_row * probe, 0.0)
    s = int(min(n_fact, max(probe, (target_s - fixed) / per_row)))
    t = run(s) if s != probe else t1
    return {"value": s / t, "unit": "rows/s", "cores": 1, "kind": "oracle",
            "sample": f"first {s} of {n_fact} fact rows of the same star schema, same plan, "
                      f"{t:.1f} s on one core of {cpu_model()} ({os.cpu_count()} cores visible)"}


def bench_batch(args, torch, datagen, rel) -> dict:
    """256 join + group-by instances of log-uniform sizes (build 1k-4M rows,
    probe 10k-50M rows, 8-100k groups; SUM(value), COUNT(*) by the build
    side's group attribute): 256 sequential rel_pipeline calls, one
    rel_pipeline_batch launch sequence and its captured graph, on the same
    resident inputs, first with default tuning, then with per-instance
    records from the autotuners (the single-plan tuner's for the sequential
    calls, the batch tuner's for the batch). Results must be identical
    throughout. With --batch-per-instance the instances above 2048 groups
    are also timed one at a time, each as a one-plan batch."""
    from paper_2508_04701_amd import autotune

    seed = datagen.SEED0 + 4
    shapes = datagen.batch_shapes(seed=seed, n_inst=args.batch_instances)
    aggs = [("sum", 1), ("count", None)]
    t0 = time.perf_counter()
    inputs = []
    n_probe = n_build = 0
    for i, s in enumerate(shapes):
        d = datagen.batch_instance(seed, i, **s)
        fact = [torch.from_numpy(d["probe_key"]).cuda(), torch.from_numpy(d["probe_val"]).cuda()]
        dims = [dict(fk=0, key=torch.from_numpy(d["build_key"]).cuda(),
                     payload=torch.from_numpy(d["build_grp"]).cuda())]
        inputs.append((fact, dims, max(1, s["n_groups"])))
        n_probe += s["n_probe"]
        n_build += s["n_build"]
    torch.cuda.synchronize()
    log(f"batch: {len(shapes)} instances, {n_build} build rows, {n_probe} probe rows "
        f"ready in {time.perf_counter() - t0:.1f} s")
    stream = torch.cuda.current_stream()

    def timed(fn, steps):
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(steps):
            fn()
        stop.record(stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / steps

    def canon(plan):
        k, a = plan.result()
        o = torch.argsort(k[0])
        return [k[0][o]] + [x[o] for x in a]

    def measure(tunings, chunk=0, batch_tunings=None):
        # the sequential calls take the single-plan tuner's records, the batch
        # the batch tuner's (each tuned on its own execution path)
        batch_tunings = tunings if batch_tunings is None else batch_tunings
        singles = [rel.PreparedPipeline(f, [], dm, [("dim", 0)], aggs, g, t)
                   for (f, dm, g), t in zip(inputs, tunings)]
        # chunk_tiles and grid are batch-wide (taken from the first plan): the
        # first plan's record keeps its other fields, not its grid, which was
        # chosen for that plan running alone
        t0b = batch_tunings[0]
        t_first = rel.tuning(chunk_tiles=chunk) if t0b is None else \
            rel.tuning(**{**{k: getattr(t0b, k) for k in autotune.FIELDS},
                          "chunk_tiles": chunk, "grid": 0})
        plans = [rel.Plan(f, [], dm, [("dim", 0)], aggs, g, t_first if i == 0 else t)
                 for i, ((f, dm, g), t) in enumerate(zip(inputs, batch_tunings))]
        batch = rel.PreparedBatch(plans)

        def sequential():
            for p in singles:
                p.launch()

        sequential()
        batch.launch()
        torch.cuda.synchronize()
        seq_ms = timed(sequential, args.batch_steps)
        batch_ms = timed(batch.launch, args.batch_steps)
        rel.profile_read()
        rel.profile_enable(True)
        batch.launch()
        torch.cuda.synchronize()
        rel.profile_enable(False)
        prof = rel.profile_read()
        batch.capture()
        batch.launch_graph()
        graph_ms = timed(batch.launch_graph, args.batch_steps)
        results = [canon(p) for p in plans]
        same = all(len(x) == len(y) and all(torch.equal(u, v) for u, v in zip(x, y))
                   for x, y in zip(results, [canon(p) for p in singles]))
        batch.release()
        out = {"sequential_ms": seq_ms, "batched_ms": batch_ms, "graph_ms": graph_ms,
               "speedup_vs_sequential": seq_ms / min(batch_ms, graph_ms),
               # one batch: its fused launches (one per LDS class) summed
               "fused_kernel_ms": prof["pipeline_fused"][0],
               "fused_launches": prof["pipeline_fused"][1],
               "breakdown_ms": {k: round(v[0], 4) for k, v in prof.items() if v[1]}}
        del singles, plans, batch
        torch.cuda.empty_cache()
        return out, results, same

    default, ref, same_default = measure([None] * len(inputs))
    log(f"batch default: {default['sequential_ms']:.1f} ms sequential, "
        f"{default['batched_ms']:.1f} ms batched, {default['graph_ms']:.1f} ms graph")

    # (--batch-per-instance) the instances above 2048 groups one at a time,
    # each as a one-plan batch with default tuning (their spilled rows go
    # through the record passes): device time summed over the batch's
    # kernel classes (HIP events around each launch, so host gaps between
    # launches do not count)
    above_2k = None
    if args.batch_per_instance:
        per_inst = []
        for (f, dm, g), shp in zip(inputs, shapes):
            if shp["n_groups"] <= 2048:
                continue
            one = rel.PreparedBatch([rel.Plan(f, [], dm, [("dim", 0)], aggs, g)])
            one.launch()
            torch.cuda.synchronize()
            rel.profile_read()
            rel.profile_enable(True)
            for _ in range(3):
                one.launch()
            torch.cuda.synchronize()
            rel.profile_enable(False)
            ms = sum(v[0] for v in rel.profile_read().values()) / 3
            one.release()
            del one
            per_inst.append([shp["n_groups"], shp["n_probe"], round(ms, 4)])
        rates = sorted(r / (ms * 1e-3) for _, r, ms in per_inst)
        above_2k = {"instances": len(per_inst),
                    "rows_per_s": {"min": rates[0], "median": rates[len(rates) // 2],
                                   "max": rates[-1]} if rates else None,
                    "per_instance": per_inst}
        if rates:
            log(f"batch: {len(per_inst)} instances above 2048 groups alone: "
                f"{rates[0] / 1e9:.2f}-{rates[-1] / 1e9:.1f} G rows/s (median "
                f"{rates[len(rates) // 2] / 1e9:.1f})")

    # autotuners: one record per size bucket, tuned on its median instance
    # (probe side cut to at most 8M rows), for the single-plan path
    # (rel_pipeline calls) and, natively, for the batched path (rel_autotune:
    # each candidate timed as a one-plan batch)
    t0 = time.perf_counter()
    cache = autotune.Cache()
    by_bucket = {}
    for i, (f, dm, g) in enumerate(inputs):
        b = autotune.plan_bucket(f[0].numel(), [dm[0]["key"].numel()], g)
        by_bucket.setdefault(b, []).append(i)
    samples = []
    for b, members in by_bucket.items():
        members.sort(key=lambda i: inputs[i][0][0].numel())
        f, dm, g = inputs[members[len(members) // 2]]
        cut = min(f[0].numel(), 8_000_000)
        sample = [f[0][:cut], f[1][:cut]]
        rec = autotune.tune_plan(lambda t: rel.PreparedPipeline(sample, [], dm, [("dim", 0)],
                                                                aggs, g, t))
        cache.put(autotune.cache_key("join_groupby", b), rec)
        samples.append(rel.Plan(sample, [], dm, [("dim", 0)], aggs, g))
    tune_s = time.perf_counter() - t0
    tunings = [autotune.tuning_for(cache, "join_groupby", f[0].numel(), [dm[0]["key"].numel()], g)
               for f, dm, g in inputs]
    t0 = time.perf_counter()
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "batch_tune.json")
        autotune.tune_batch_plans(samples, path)
        batch_tunings = [autotune.lookup(path, rel.Plan(f, [], dm, [("dim", 0)], aggs, g))
                         for f, dm, g in inputs]
    tune_batch_s = time.perf_counter() - t0
    del samples
    best = None
    for chunk in args.batch_chunks:
        res, got, same = measure(tunings, chunk, batch_tunings)
        same = same and all(all(torch.equal(u, v) for u, v in zip(x, y)) for x, y in zip(got, ref))
        res["chunk_tiles"] = chunk
        res["identical_results"] = same
        log(f"batch tuned (chunk {chunk}): {res['sequential_ms']:.1f} ms sequential, "
            f"{res['batched_ms']:.1f} ms batched, {res['graph_ms']:.1f} ms graph, same {same}")
        if best is None or min(res["batched_ms"], res["graph_ms"]) < \
                min(best["batched_ms"], best["graph_ms"]):
            best = res
    if args.tune_cache_out:
        cache.save(args.tune_cache_out)
    # the top-level figures come from the faster configuration, default or
    # tuned, each against its own sequential calls
    tuned = best
    top, top_from = (default, "default") if min(default["batched_ms"], default["graph_ms"]) <= \
        min(tuned["batched_ms"], tuned["graph_ms"]) else (tuned, "tuned")
    alg = 12 * n_probe + 8 * n_build
    best_ms = min(top["batched_ms"], top["graph_ms"])
    return {
        "workload": f"{len(shapes)} join+group-by instances, log-uniform build 1k-4M, "
                    f"probe 10k-50M, groups 8-100k",
        "instances": len(shapes), "probe_rows": n_probe, "build_rows": n_build,
        "default": {**default, "identical_results": same_default},
        **({"above_2k_groups_alone": above_2k} if above_2k else {}),
        "tuned": tuned,
        "autotune": {"buckets": len(by_bucket), "seconds": tune_s, "batch_seconds": tune_batch_s},
        "top_level_from": top_from,
        "batched_rows_per_s": n_probe / (best_ms * 1e-3),
        "sequential_rows_per_s": n_probe / (top["sequential_ms"] * 1e-3),
        "speedup_vs_sequential": top["sequential_ms"] / best_ms,
        "identical_results": same_default and tuned["identical_results"],
        "algorithmic_bytes": alg, "hbm_frac_step": alg / (best_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
    }


def bench_ops(args, torch, datagen, rel) -> dict:
    """Each standalone operator against its own HBM roofline, with the bytes
    the operation must move (inputs read once, outputs written once; random
    hash-table traffic is the method's cost, not counted): rel_filter on the
    star schema's 600M-row date column (date < 767); rel_hash_join and
    rel_groupby_agg on the skewed workload (100M unique int64 build keys,
    400M Zipf(1) probe keys, every probe matching once; about 10M groups of
    an int64 probe-side column). Device time per kernel class from HIP
    events over the timed launches."""
    reps = args.ops_reps

    def kernel_ms(fn):
        fn()
        torch.cuda.synchronize()
        rel.profile_read()
        rel.profile_enable(True)
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        rel.profile_enable(False)
        return {k: v[0] / reps for k, v in rel.profile_read().items() if v[1]}

    def line(ms, nbytes, **kw):
        gbs = nbytes / (ms * 1e-3) / 1e9
        return {**kw, "kernel_ms": ms, "algorithmic_bytes": nbytes, "achieved_gbs": gbs,
                "frac": gbs / HBM_PEAK_GBS}

    res = {}
    n = args.n_fact
    date = torch.from_numpy(datagen.uniform(datagen.SEED0 + 2, 12, 0, 2557, n, np.int32)).cuda()
    ids = torch.empty(n, dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = rel.workspace(rel.filter_ws(n))
    k = kernel_ms(lambda: rel.filter_async([date], [(0, "lt", 767)], ids, count, ws))
    passing = int(count.item())
    res["filter"] = line(k["filter"], 4 * n + 4 * passing, rows=n, passing=passing,
                         workload=f"int32 date[{n}] < 767 -> ascending row ids")
    del date, ids, ws
    torch.cuda.empty_cache()

    t0 = time.perf_counter()
    sk = datagen.skewed(n_build=args.ops_build, n_probe=args.ops_probe, n_groups=args.ops_groups)
    dev = {c: torch.from_numpy(v).cuda() for c, v in sk.items()}
    del sk
    log(f"ops: skewed workload ready in {time.perf_counter() - t0:.1f} s")
    nb, npr = dev["build_key"].numel(), dev["probe_key"].numel()
    ws = rel.workspace(rel.hash_join_ws(torch.int64, nb))
    ob = torch.empty(npr, dtype=torch.int32, device="cuda")
    op = torch.empty(npr, dtype=torch.int32, device="cuda")
    k = kernel_ms(lambda: rel.hash_join_async(dev["build_key"], dev["probe_key"], ob, op, count, ws))
    pairs = int(count.item())
    res["hash_build"] = line(k["map_build"], 8 * nb, rows=nb,
                             workload=f"{nb} unique int64 keys -> open-addressing table "
                                      "(partitioned: ranges built in LDS)")
    res["hash_probe"] = line(k["map_probe"], 8 * npr + 8 * pairs, rows=npr, pairs=pairs,
                             workload=f"{npr} Zipf(1) int64 probe keys -> (build, probe) row-id pairs")
    res["hash_join_fill_ms"] = k.get("fill", 0.0)

    # join -> group-by as one composite step: the pairs' probe row ids feed
    # the group-by as a gather-on-read selection of the probe side's group
    # and payload columns (every probe row matches once here)
    aggs2 = [("sum", 0), ("count", None)]
    mg = args.ops_groups
    gk = [torch.empty(mg, dtype=torch.int64, device="cuda")]
    ga = [torch.empty(mg, dtype=torch.int64, device="cuda") for _ in aggs2]
    gcount = torch.zeros(1, dtype=torch.int64, device="cuda")
    sel = op[:pairs]
    wsg = rel.workspace(rel.groupby_ws([torch.int64], aggs2, pairs, mg))

    def composite():
        rel.hash_join_async(dev["build_key"], dev["probe_key"], ob, op, count, ws)
        rel.groupby_agg_async([dev["probe_grp"]], [dev["probe_val"]], aggs2, gk, ga, gcount, mg,
                              wsg, key_idx=sel, val_idx=sel)

    composite()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        composite()
    stop.record()
    torch.cuda.synchronize()
    cms = start.elapsed_time(stop) / reps
    cbytes = 8 * nb + 8 * npr + 16 * pairs + int(gcount.item()) * 24
    res["join_groupby_composite"] = {
        "ms": cms, "rows": npr, "rows_per_s": npr / (cms * 1e-3), "groups": int(gcount.item()),
        "algorithmic_bytes": cbytes,
        "frac": cbytes / (cms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "workload": f"rel_hash_join ({nb} unique int64 build keys, {npr} Zipf(1) probes) then "
                    "rel_groupby_agg of the matched rows' int64 group column (~10M groups), "
                    "SUM/COUNT of the payload, selected through the probe row ids"}
    del ws, wsg, gk, ga, sel
    torch.cuda.empty_cache()
    # the single-pass build (one device-scope CAS per key after filling the
    # table) beside it
    single = rel.tuning(fanout=-1)
    ws = rel.workspace(rel.hash_join_ws(torch.int64, nb, single))
    k = kernel_ms(lambda: rel.hash_join_async(dev["build_key"], dev["probe_key"], ob, op, count, ws,
                                              t=single))
    res["hash_build_single_pass"] = line(k["map_build"] + k.get("fill", 0.0), 8 * nb, rows=nb,
                                         workload=f"{nb} unique int64 keys, table fill + one CAS "
                                                  "per key")
    del ws, ob, op
    torch.cuda.empty_cache()

    res.update(bench_bloom(args, torch, datagen, rel, kernel_ms, line))
    res.update(bench_strings(args, torch, datagen, rel, kernel_ms, line))
    res.update(bench_topn(args, torch, datagen, rel, kernel_ms, line))

    aggs = [("sum", 0), ("count", None), ("avg", 0), ("min", 0), ("max", 0)]
    mg = args.ops_groups
    out_keys = [torch.empty(mg, dtype=torch.int64, device="cuda")]
    out_aggs = [torch.empty(mg, dtype=torch.float64 if a == "avg" else torch.int64, device="cuda")
                for a, _ in aggs]
    wl = (f"{npr} rows, int64 Zipf-skewed key over {mg} values, "
          "SUM/COUNT/AVG/MIN/MAX of an int64 column")
    # the single-pass hash aggregation (every row updates the global table)
    # beside the default, which radix-partitions tables of this size
    single = rel.tuning(fanout=-1)
    ws = rel.workspace(rel.groupby_ws([torch.int64], aggs, npr, mg, single))
    k = kernel_ms(lambda: rel.groupby_agg_async([dev["probe_grp"]], [dev["probe_val"]], aggs,
                                                out_keys, out_aggs, count, mg, ws, t=single))
    res["group_by_single_pass"] = line(k["group_agg"], 16 * npr, rows=npr, workload=wl)
    del ws
    torch.cuda.empty_cache()
    ws = rel.workspace(rel.groupby_ws([torch.int64], aggs, npr, mg))
    k = kernel_ms(lambda: rel.groupby_agg_async([dev["probe_grp"]], [dev["probe_val"]], aggs,
                                                out_keys, out_aggs, count, mg, ws))
    groups = int(count.item())
    part_ms = k.get("group_partition", 0.0)
    res["group_by"] = line(k["group_agg"] + part_ms, 16 * npr, rows=npr, groups=groups,
                           partition_ms=part_ms, aggregate_ms=k["group_agg"], workload=wl)
    del ws
    torch.cuda.empty_cache()
    # the autotuner's group-by record for this size bucket (fan-out, first
    # scatter's LDS table), every candidate checked for identical groups
    from paper_2508_04701_amd import autotune
    rec = autotune.tune_groupby([dev["probe_grp"]], [dev["probe_val"]], aggs, mg)
    res["group_by_autotune"] = {"bucket": autotune.bucket(npr, 0, mg), "tuning": rec["tuning"],
                                "ms": rec["ms"], "candidates_ms": rec["candidates"]}
    res["finalize"] = line(k["group_finalize"], groups * (8 + 8 * len(aggs)), groups=groups,
                           workload="occupied group slots -> key and aggregate columns "
                                    "(includes the replica merge)")
    return res


def bench_bloom(args, torch, datagen, rel, kernel_ms, line) -> dict:
    """Predicate transfer on a join with few partners: --bloom-build unique
    int64 build keys (1M by default), --bloom-probe probe keys (400M) of which
    5% are build keys and the rest draws from the whole int64 range. The hash join with and without the Bloom filter
    in front of its table walk, and the filter alone (rel_bloom_filter: the
    probe rows that may have a partner)."""
    seed = datagen.SEED0 + 6
    nb, npr = args.bloom_build, args.bloom_probe
    build = datagen.unique_i64(seed, 40, nb)
    hit = datagen.uniform(seed, 41, 0, 100, npr, np.int32) < 5
    pick = datagen.uniform(seed, 42, 0, nb, npr, np.int64)
    probe = datagen.raw_u64(seed, 43, npr).view(np.int64)
    probe[hit] = build[pick[hit]]
    del hit, pick
    bk, pk = torch.from_numpy(build).cuda(), torch.from_numpy(probe).cuda()
    del build, probe
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    cap = npr // 10
    ob = torch.empty(cap, dtype=torch.int32, device="cuda")
    op = torch.empty(cap, dtype=torch.int32, device="cuda")
    out = {}
    wl = f"{nb} unique int64 build keys, {npr} probe keys, 5% with a partner"
    for name, t in (("join_low_match", None), ("join_low_match_bloom", rel.tuning(flags=rel.TUNE_BLOOM))):
        ws = rel.workspace(rel.hash_join_ws(torch.int64, nb, t))
        k = kernel_ms(lambda: rel.hash_join_async(bk, pk, ob, op, count, ws, t=t))
        ms = sum(k.values())
        out[name] = line(ms, 8 * nb + 8 * npr + 8 * int(count.item()), rows=npr,
                         pairs=int(count.item()), rows_per_s=npr / (ms * 1e-3),
                         breakdown_ms={kk: round(v, 4) for kk, v in k.items()},
                         workload=wl + (", Bloom filter in front of the table" if t else ""))
        del ws
    f = rel.bloom_build(bk)
    ids = torch.empty(npr, dtype=torch.int32, device="cuda")
    ws = rel.workspace(rel.filter_ws(npr))
    k = kernel_ms(lambda: rel.bloom_filter_async(pk, f, ids, count, ws))
    kept = int(count.item())
    out["bloom_filter"] = line(k["filter"], 8 * npr + 4 * kept, rows=npr, kept=kept,
                               filter_bytes=int(f.numel()), rows_per_s=npr / (k["filter"] * 1e-3),
                               workload=f"{npr} int64 probe keys through a 16-bit-per-key Bloom "
                                        f"filter of {nb} build keys -> ascending row ids")
    out["join_low_match_bloom"]["speedup_vs_plain"] = (
        out["join_low_match"]["kernel_ms"] / out["join_low_match_bloom"]["kernel_ms"])
    del bk, pk, ob, op, ids, ws, f
    torch.cuda.empty_cache()
    return out


def bench_strings(args, torch, datagen, rel, kernel_ms, line) -> dict:
    """Group-by on a string key (a stand-in for string-keyed ClickBench
    group-bys; the suite itself is not used): a dictionary of 1M distinct
    lowercase strings of 8-48 bytes, rows drawing their string by Zipf(1)
    rank over it, COUNT(*) and SUM of an int64 column - dictionary-encoded
    (int32 codes) over 100M rows, and materialised in the Arrow layout
    (offsets + bytes) over 20M rows."""
    seed = datagen.SEED0 + 7
    nd = args.str_dict
    lens = datagen.uniform(seed, 50, 8, 49, nd, np.int64)
    offsets = np.zeros(nd + 1, np.int64)
    offsets[1:] = np.cumsum(lens)
    data = datagen.uniform(seed, 51, 97, 123, int(offsets[-1]), np.uint8)
    out = {}
    aggs = [("count", None), ("sum", 0)]
    for name, n, plain in (("groupby_string_dict", args.str_rows, False),
                           ("groupby_string_plain", args.str_rows // 5, True)):
        codes = (datagen.zipf_ranks(seed, 52, nd, 1.0, n) - 1).astype(np.int32)
        val = datagen.uniform(seed, 53, 0, 1_000_000, n, np.int64)
        if plain:
            lens_r = lens[codes]
            off_r = np.zeros(n + 1, np.int64)
            off_r[1:] = np.cumsum(lens_r)
            # the rows' bytes, string by string (a gather of byte ranges)
            starts = np.repeat(offsets[:-1][codes] - off_r[:-1], lens_r)
            data_r = data[np.arange(int(off_r[-1]), dtype=np.int64) + starts]
            del starts, lens_r
            doff, ddata, dcodes = (torch.from_numpy(off_r).cuda(), torch.from_numpy(data_r).cuda(),
                                   None)
            nbytes = 8 * (n + 1) + int(off_r[-1]) + 8 * n
            del off_r, data_r
        else:
            doff, ddata = torch.from_numpy(offsets).cuda(), torch.from_numpy(data).cuda()
            dcodes = torch.from_numpy(codes).cuda()
            nbytes = 4 * n + 8 * n  # codes and values; the dictionary stays in the caches
        dval = torch.from_numpy(val).cuda()
        del codes, val
        mg = nd
        ws = rel.workspace(rel.groupby_str_ws(aggs, mg, 0 if plain else nd))
        st = rel.strings(doff, ddata, dcodes)
        cv = rel._arr(rel.Column, [rel.column(dval)])
        rows = torch.empty(mg, dtype=torch.int32, device="cuda")
        oa = [torch.empty(mg, dtype=torch.int64, device="cuda") for _ in aggs]
        oap = rel._arr(rel.ctypes.c_void_p, [o.data_ptr() for o in oa])
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")

        def call():
            rel._check(rel.lib().rel_groupby_str(rel.ctypes.byref(st), None, cv, 1, rel._aggs(aggs),
                                                 len(aggs), rel._addr(rows), None, oap, mg,
                                                 rel._addr(cnt), mg, rel._addr(ws), ws.numel(),
                                                 rel._stream()))

        k = kernel_ms(call)
        ms = sum(k.values())
        out[name] = line(ms, nbytes, rows=n, groups=int(cnt.item()), rows_per_s=n / (ms * 1e-3),
                         breakdown_ms={kk: round(v, 4) for kk, v in k.items()},
                         workload=f"{n} rows, Zipf(1) over {nd} distinct strings of 8-48 bytes, "
                                  + ("Arrow offsets + bytes" if plain else "int32 dictionary codes")
                                  + ", COUNT(*), SUM(int64)")
        del doff, ddata, dcodes, dval, ws, rows, oa
        torch.cuda.empty_cache()
    return out


def bench_topn(args, torch, datagen, rel, kernel_ms, line) -> dict:
    """ORDER BY ... LIMIT over a large result table: 10M groups (int64 key,
    int64 SUM with ties), the top 100 and the top 1000 by SUM descending, ties
    by key, then the rows materialised by rel_gather."""
    seed = datagen.SEED0 + 8
    n = args.topn_rows
    key = torch.from_numpy(datagen.unique_i64(seed, 60, n)).cuda()
    val = torch.from_numpy(datagen.uniform(seed, 61, 0, 1_000_000, n, np.int64)).cuda()
    out = {}
    for limit in (100, 1000):
        pos = torch.empty(limit, dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        ws = rel.workspace(rel.topn_ws(n, limit))
        k = kernel_ms(lambda: rel.topn_async(val, [key], limit, pos, cnt, ws, desc=True))
        dst = [torch.empty(limit, dtype=torch.int64, device="cuda") for _ in range(2)]
        g = kernel_ms(lambda: rel.gather_async([key, val], pos, dst))
        out[f"top_{limit}"] = line(k["top_n"], 16 * n, rows=n, limit=limit,
                                   gather_ms=g["gather"], rows_per_s=n / (k["top_n"] * 1e-3),
                                   workload=f"{n} rows (int64 key, int64 value), top {limit} by "
                                            "value descending, ties by key; then the rows gathered")
        del pos, ws, dst
    del key, val
    torch.cuda.empty_cache()
    return out


def bench_out_of_core(args, torch, datagen, rel) -> dict:
    """The star-schema plan (hash-table dims) with the 600M-row fact table in
    pinned host memory, streamed through the device in chunks while the
    previous chunk is aggregated (rel_pipeline_stream), beside the plain
    host-to-device copy of the same bytes (the link's ceiling) and the result
    of the resident plan."""
    seed = datagen.SEED0 + 2
    n = args.n_fact
    d = datagen.star_schema(seed=seed, n_fact=n)
    t0 = time.perf_counter()
    host = [torch.from_numpy(d[k]).pin_memory() for k in ("fk_a", "fk_b", "date", "price", "flag")]
    log(f"out-of-core: {n} fact rows pinned in {time.perf_counter() - t0:.1f} s")
    dims = [dict(fk=0, key=torch.from_numpy(d["dim_a_key"]).cuda(), payload=None),
            dict(fk=1, key=torch.from_numpy(d["dim_b_key"]).cuda(),
                 payload=torch.from_numpy(d["dim_b_region"]).cuda())]
    del d
    nbytes = sum(c.numel() * c.element_size() for c in host)
    stream = torch.cuda.current_stream()
    # the link's ceiling: one copy of every column to the device
    dst = [torch.empty_like(c, device="cuda") for c in host]
    for a, b in zip(dst, host):
        a.copy_(b, non_blocking=True)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for a, b in zip(dst, host):
        a.copy_(b, non_blocking=True)
    stop.record(stream)
    torch.cuda.synchronize()
    copy_ms = start.elapsed_time(stop)
    resident = rel.PreparedPipeline(dst, TERMS, dims, KEYS, AGGS, 128,
                                    rel.tuning(flags=rel.TUNE_NO_DIRECT))
    resident.launch()
    want = resident.result()
    del resident, dst
    torch.cuda.empty_cache()
    res = {"workload": f"star schema, {n} fact rows ({nbytes / 1e9:.1f} GB) in pinned host memory, "
                       "hash-table dims", "h2d_copy_ms": copy_ms,
           "h2d_gbs": nbytes / (copy_ms * 1e-3) / 1e9, "chunks": {}}
    for chunk in args.ooc_chunks:
        plan = rel.StreamedPipeline(host, TERMS, dims, KEYS, AGGS, 128, chunk,
                                    rel.tuning(flags=rel.TUNE_NO_DIRECT))
        plan.launch()
        got = plan.result()
        same = all(torch.equal(x, y) for x, y in zip(sorted_groups(torch, *got),
                                                     sorted_groups(torch, *want)))
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(args.ooc_steps):
            plan.launch()
        stop.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / args.ooc_steps
        res["chunks"][str(chunk)] = {"ms": ms, "rows_per_s": n / (ms * 1e-3),
                                     "gbs": nbytes / (ms * 1e-3) / 1e9,
                                     "frac_of_h2d": copy_ms / ms, "identical_to_resident": same}
        log(f"out-of-core: chunk {chunk}: {ms:.1f} ms ({copy_ms:.1f} ms to copy), same {same}")
        del plan
        torch.cuda.empty_cache()
    return res


def sorted_groups(torch, keys, aggs):
    o = torch.argsort(keys[0].long() * 4 + keys[1].long())
    return [k[o] for k in keys] + [a[o] for a in aggs]


SERVE_AGGS = [("sum", 3), ("count", None)]


class QueryPool:
    """Plans of the served queries, recycled: per grouping attribute a fixed
    set of plans with device and pinned host outputs; query i takes a free one
    of its attribute and sets its date range (the server copies the plan at
    submission), and gives it back when it completes. With none free the
    query waits on the client (its latency still counts from its arrival)."""

    def __init__(self, rel, serve, fact, dims, groups, attr, lo, hi, per_attr):
        self.attr, self.lo, self.hi = attr, lo, hi
        self.free = {}
        for a in range(len(dims)):
            self.free[a] = []
            for _ in range(per_attr):
                plan = rel.Plan(fact, [(2, "range", 0, 1)], [dims[a]], [("dim", 0)], SERVE_AGGS,
                                groups[a])
                self.free[a].append((plan, serve.HostResult(plan)))
        self.busy = {}

    def make(self, i):
        a = int(self.attr[i])
        if not self.free[a]:
            return None
        plan, host = self.free[a].pop()
        plan._preds[0].lo = int(self.lo[i])
        plan._preds[0].hi = int(self.hi[i])
        self.busy[i] = (a, plan, host)
        return plan, host

    def done(self, i, completion):
        a, plan, host = self.busy.pop(i)
        self.free[a].append((plan, host))


def bench_serve(args, torch, datagen, rel) -> dict:
    """Queries over a resident 200M-row star schema: date range of 1-50%
    selectivity, join with the dim holding the grouping attribute (dim B
    region: 25 groups, dim B city: 5,000, dim A segment: 1,000,000),
    SUM(price) and COUNT(*). A seeded Poisson trace at multiples of the
    measured one-at-a-time capacity is replayed against the server serving
    one query at a time and with continuous batching."""
    from paper_2508_04701_amd import serve

    seed = datagen.SEED0 + 5
    n_fact = args.serve_rows
    t0 = time.perf_counter()
    d = datagen.star_schema(seed=seed, n_fact=n_fact)
    nb, na = len(d["dim_b_key"]), len(d["dim_a_key"])
    city = (datagen.permutation(seed, 70, nb) % 5_000).astype(np.int32)
    segment = (datagen.permutation(seed, 71, na) % 1_000_000).astype(np.int32)
    cols = {k: torch.from_numpy(v).cuda() for k, v in d.items()}
    fact = [cols[k] for k in ("fk_a", "fk_b", "date", "price", "flag")]
    dims = [dict(fk=1, key=cols["dim_b_key"], payload=cols["dim_b_region"]),
            dict(fk=1, key=cols["dim_b_key"], payload=torch.from_numpy(city).cuda()),
            dict(fk=0, key=cols["dim_a_key"], payload=torch.from_numpy(segment).cuda())]
    groups = [25, 5_000, 1_000_000]
    del d
    nq = args.serve_queries
    u = (datagen.raw_u64(seed, 72, nq) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    w = np.rint((0.01 + 0.49 * u) * 2557).astype(np.int64)
    v = (datagen.raw_u64(seed, 74, nq) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    lo = np.floor(v * (2557 - w + 1)).astype(np.int64)
    attr = (datagen.raw_u64(seed, 75, nq) % np.uint64(3)).astype(np.int64)
    hi = lo + w
    pool = QueryPool(rel, serve, fact, dims, groups, attr, lo, hi, args.serve_pool)
    torch.cuda.synchronize()
    log(f"serve: {n_fact} resident fact rows, {nq} queries, ready in "
        f"{time.perf_counter() - t0:.1f} s")
    arena_bytes = args.serve_arena_gb << 30
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")

    modes = {"one_at_a_time": dict(max_slots=1, max_batch=1, lanes=1),
             "continuous": dict(max_slots=64, max_batch=16, lanes=args.serve_lanes,
                                open_lane_at=args.serve_open_at)}

    def run(mode, arrivals, count):
        srv = serve.Server(arena_bytes, arena_ptr=arena.data_ptr(), **modes[mode])
        out = serve.replay(srv, pool.make, arrivals[:count], on_done=pool.done)
        st = srv.stats()
        srv.close()
        out.pop("tickets")
        out["rows_per_s"] = count * n_fact / out["wall_s"]
        out["batches"] = st["batches"]
        return out

    # capacity: a burst served one query at a time, warm
    run("one_at_a_time", np.zeros(32), 32)
    burst = run("one_at_a_time", np.zeros(args.serve_calib), args.serve_calib)
    capacity = args.serve_calib / burst["wall_s"]
    log(f"serve: one-at-a-time capacity {capacity:.1f} queries/s")
    result = {"workload": f"{n_fact}-row resident star schema, date range 1-50% selectivity, "
                          "group by dim B region (25) / city (5k) / dim A segment (1M), "
                          "SUM(price), COUNT(*); seeded Poisson arrivals",
              "fact_rows": n_fact, "capacity_one_at_a_time_qps": capacity, "rates": []}
    for x in args.serve_rates:
        count = nq if x == 0.8 else min(nq, args.serve_sweep_queries)
        arrivals = serve.poisson_arrivals(seed, count, x * capacity)
        point = {"x_capacity": x, "qps": x * capacity, "queries": count}
        for mode in modes:
            point[mode] = run(mode, arrivals, count)
            log(f"serve: {x}x {mode}: p50 {point[mode]['p50_ms']:.2f} ms, p99 "
                f"{point[mode]['p99_ms']:.2f} ms, {point[mode]['rows_per_s'] / 1e9:.1f} G rows/s")
        result["rates"].append(point)
    return result


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-fact", type=int, default=600_000_000)
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stream-reps", type=int, default=5)
    ap.add_argument("--no-c1", action="store_true", help="skip the 64k x 1M join + group-by")
    ap.add_argument("--c1-reps", type=int, default=20)
    ap.add_argument("--tables", choices=["hash", "direct"], default=None,
                    help="only time the star-schema step with these dim tables (profiling)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-instances section")
    ap.add_argument("--batch-only", action="store_true")
    ap.add_argument("--batch-instances", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--batch-chunks", type=int, nargs="*", default=[0, 2])
    ap.add_argument("--batch-per-instance", action="store_true",
                    help="also time each batched instance above 2048 groups alone")
    ap.add_argument("--tune-cache-out", default=None,
                    help="write the autotuner records of the batched section to this JSON file")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving section")
    ap.add_argument("--no-ops", action="store_true", help="skip the standalone-operator section")
    ap.add_argument("--ops-only", action="store_true")
    ap.add_argument("--ops-reps", type=int, default=3)
    ap.add_argument("--ops-build", type=int, default=100_000_000)
    ap.add_argument("--ops-probe", type=int, default=400_000_000)
    ap.add_argument("--ops-groups", type=int, default=10_000_000)
    ap.add_argument("--bloom-build", type=int, default=1_000_000)
    ap.add_argument("--bloom-probe", type=int, default=400_000_000)
    ap.add_argument("--str-dict", type=int, default=1_000_000)
    ap.add_argument("--str-rows", type=int, default=100_000_000)
    ap.add_argument("--topn-rows", type=int, default=10_000_000)
    ap.add_argument("--no-ooc", action="store_true", help="skip the out-of-core section")
    ap.add_argument("--ooc-only", action="store_true")
    ap.add_argument("--ooc-steps", type=int, default=2)
    ap.add_argument("--ooc-chunks", type=int, nargs="*", default=[2048 * 4096, 2048 * 16384])
    ap.add_argument("--serve-only", action="store_true")
    ap.add_argument("--serve-rows", type=int, default=200_000_000)
    ap.add_argument("--serve-queries", type=int, default=2000)
    ap.add_argument("--serve-sweep-queries", type=int, default=400)
    ap.add_argument("--serve-calib", type=int, default=100)
    ap.add_argument("--serve-pool", type=int, default=96)
    ap.add_argument("--serve-arena-gb", type=int, default=64)
    ap.add_argument("--serve-rates", type=float, nargs="*", default=[0.5, 0.8, 1.2, 2.0])
    ap.add_argument("--serve-lanes", type=int, default=2,
                    help="continuous mode: batches in flight at once")
    ap.add_argument("--serve-open-at", type=int, default=1,
                    help="continuous mode: backlog that opens a further lane while one is busy")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (for scaling the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the relational path here runs on a single MI355X "
              "(multi-GPU sharding is described, not built). Run with --gpus 1.", file=sys.stderr)
        return 2

    import torch

    from paper_2508_04701_amd import datagen, rel

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "launches": 3}), flush=True)
        return 0
    if args.batch_only:
        print(json.dumps({"batch": bench_batch(args, torch, datagen, rel)}), flush=True)
        return 0
    if args.ops_only:
        print(json.dumps({"ops": bench_ops(args, torch, datagen, rel)}), flush=True)
        return 0
    if args.serve_only:
        print(json.dumps({"serving": bench_serve(args, torch, datagen, rel)}), flush=True)
        return 0
    if args.ooc_only:
        print(json.dumps({"out_of_core": bench_out_of_core(args, torch, datagen, rel)}), flush=True)
        return 0
    seed = datagen.SEED0 + 2 if args.seed is None else args.seed
    n = args.n_fact

    t0 = time.perf_counter()
    d = datagen.star_schema(seed=seed, n_fact=n)
    log(f"generated {n} fact rows in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    dev = {k: torch.from_numpy(v).to("cuda") for k, v in d.items()}
    torch.cuda.synchronize()
    log(f"uploaded in {time.perf_counter() - t0:.1f} s")

    fact = [dev["fk_a"], dev["fk_b"], dev["date"], dev["price"], dev["flag"]]
    dims = [dict(fk=0, key=dev["dim_a_key"], payload=None),
            dict(fk=1, key=dev["dim_b_key"], payload=dev["dim_b_region"])]
    alg_bytes = FACT_BYTES_PER_ROW * n
    if args.tables:
        t = rel.tuning(flags=rel.TUNE_NO_DIRECT) if args.tables == "hash" else None
        r = star_run(args, torch, rel, fact, dims, t)
        r.pop("result")
        print(json.dumps({"tables": args.tables, **r}), flush=True)
        return 0
    # headline: both dims in open-addressing hash tables; beside it the
    # same plan with the dense dim keys in direct tables
    hashed = star_run(args, torch, rel, fact, dims, rel.tuning(flags=rel.TUNE_NO_DIRECT))
    direct = star_run(args, torch, rel, fact, dims, None)
    same = all(torch.equal(x, y) for x, y in zip(hashed.pop("result"), direct.pop("result")))
    stream = stream_ceiling(args, torch, rel, fact)
    fused_avg_ms = hashed["fused_kernel_ms"]
    achieved_gbs = alg_bytes / (fused_avg_ms * 1e-3) / 1e9
    ms_per_step = hashed["ms_per_step"]

    out = {
        "metric": METRIC,
        "value": n / (ms_per_step * 1e-3),
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "star schema: 600M-row fact, date < 767, join dim A (1.5M) "
                               "and dim B (10k) through open-addressing hash tables, "
                               "group by (region, flag), SUM/COUNT/AVG/MIN/MAX(price)"
                   if n == 600_000_000 else f"star schema with {n} fact rows, hash-table dims",
                   "fact_rows": n, "groups": hashed["groups"], "seed": seed,
                   "dim_tables": "hash (rel_tuning.flags = REL_TUNE_NO_DIRECT)"},
        "hbm_frac_step": alg_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "breakdown_ms_per_step": hashed["breakdown_ms_per_step"],
        "roofline": {"bound": "hbm", "kernel": "pipeline_fused", "achieved": achieved_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved_gbs / HBM_PEAK_GBS,
                     "frac_of_stream": achieved_gbs / stream["achieved_gbs"],
                     "kernel_ms": fused_avg_ms, "algorithmic_bytes": alg_bytes,
                     "traffic": measured_traffic(n, TRAFFIC_PROFILE)},
        "stream_read": stream,
        "direct_tables": {
            "workload": "the same plan with both dims in direct tables (dense unique keys: "
                        "dim A a range test, dim B a byte array)",
            "ms_per_step": direct["ms_per_step"], "rows_per_s": n / (direct["ms_per_step"] * 1e-3),
            "fused_kernel_ms": direct["fused_kernel_ms"],
            "frac": alg_bytes / (direct["fused_kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "traffic": measured_traffic(n, TRAFFIC_PROFILE_DIRECT),
            "breakdown_ms_per_step": direct["breakdown_ms_per_step"],
            "identical_results": same},
    }
    if not args.no_c1:
        out["join_groupby_64k_1m"] = bench_c1(args, torch, datagen, rel)
    if not args.no_cpu_baseline:
        host = {k: v for k, v in d.items()}
        out["cpu_baseline"] = cpu_baseline(host, n, args.cpu_seconds)
        del host
    if not args.no_batch:
        del fact, dims, dev, d
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        out["batch"] = bench_batch(args, torch, datagen, rel)
    if not args.no_serve:
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        out["serving"] = bench_serve(args, torch, datagen, rel)
    if not args.no_ops:
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        out["ops"] = bench_ops(args, torch, datagen, rel)
    if not args.no_ooc:
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        out["out_of_core"] = bench_out_of_core(args, torch, datagen, rel)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
