"""GPU parity of batched plans (rel_pipeline_batch and its captured graph):
every instance of a batch must equal the same plan run alone through
rel_pipeline and the oracle, exactly (AVG bit for bit), whatever the work
split (chunk size, grid) and across graph replays."""

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import announce, assert_groups, canon_groups, dev
from paper_2508_04701_amd import datagen, rel

pytestmark = pytest.mark.gpu

AGGS = [("sum", 1), ("count", None), ("avg", 1), ("min", 1), ("max", 1)]


def join_instances(seed, n_inst, build_range, probe_range, group_range):
    shapes = datagen.batch_shapes(seed=seed, n_inst=n_inst, build_range=build_range,
                                  probe_range=probe_range, group_range=group_range)
    return [dict(shape=s, **datagen.batch_instance(seed, i, **s)) for i, s in enumerate(shapes)]


def join_spec(inst):
    """(fact, terms, dims, keys, aggs, max_groups) of a join + group-by
    instance: probe side as the fact table, build side as the dim."""
    fact = [inst["probe_key"], inst["probe_val"]]
    dims = [dict(fk=0, key=inst["build_key"], payload=inst["build_grp"])]
    return fact, [], dims, [("dim", 0)], AGGS, max(1, inst["shape"]["n_groups"])


def device_plan(spec, t=None):
    fact, terms, dims, keys, aggs, max_groups = spec
    ddims = [dict(fk=x["fk"], key=dev(x["key"]),
                  payload=None if x.get("payload") is None else dev(x["payload"])) for x in dims]
    return rel.Plan([dev(c) for c in fact], terms, ddims, keys, aggs, max_groups, t)


def oracle_of(spec):
    fact, terms, dims, keys, aggs, _ = spec
    return oracle.pipeline(fact, terms, dims, keys, aggs)


def assert_same(a, b, what):
    ka, aa = canon_groups(*a)
    kb, ab = canon_groups(*b)
    assert len(aa[0]) == len(ab[0]), f"{what}: {len(aa[0])} vs {len(ab[0])} groups"
    for x, y in zip(ka + aa, kb + ab):
        assert np.array_equal(x, y), what


def run_batch(specs, t0=None, graph=False):
    plans = [device_plan(s, t0 if i == 0 else None) for i, s in enumerate(specs)]
    b = rel.PreparedBatch(plans)
    if graph:
        b.capture()
        b.launch_graph()
    else:
        b.launch()
    torch.cuda.synchronize()
    return b


def test_batch_join_instances_match_single_calls_and_oracle():
    announce("batch join instances", 24)
    insts = join_instances(101, 24, (100, 40_000), (1_000, 400_000), (8, 5_000))
    # edge instances: no probe rows, one build row, no build rows
    insts[3]["probe_key"] = insts[3]["probe_key"][:0]
    insts[3]["probe_val"] = insts[3]["probe_val"][:0]
    insts[5].update(build_key=np.array([7], np.int32), build_grp=np.array([2], np.int32))
    insts[9].update(build_key=np.zeros(0, np.int32), build_grp=np.zeros(0, np.int32))
    specs = [join_spec(i) for i in insts]
    b = run_batch(specs)
    for i, (spec, plan) in enumerate(zip(specs, b.plans)):
        got = plan.result()
        fact, terms, dims, keys, aggs, mg = spec
        single = rel.pipeline([dev(c) for c in fact], terms,
                              [dict(fk=0, key=dev(dims[0]["key"]), payload=dev(dims[0]["payload"]))],
                              keys, aggs, mg)
        assert_same(got, single, f"instance {i}: batch vs single call")
        assert_groups(got, oracle_of(spec), aggs, f"instance {i}")


def mixed_specs(seed, n):
    """Plans of one two-dim shape (an int32 membership dim, then an int32 dim
    with a payload) that differ in everything else: sizes (empty included),
    duplicate dim keys, predicates, group keys (none, fact, dim, both) and
    aggregates."""
    r = np.random.default_rng(seed)
    specs = []
    key_sets = [[("dim", 1)], [("fact", 2)], [], [("dim", 1), ("fact", 2)]]
    agg_sets = [AGGS, [("count", None)], [("sum", 1), ("max", 1)], [("min", 1), ("avg", 1)]]
    for i in range(n):
        nf = [0, 1, 2047, 2049, 50_000, 123_457][i % 6]
        nd0 = [0, 5, 300, 4_000][i % 4]
        nd1 = [1, 64, 2_500][i % 3]
        dup = i % 2 == 1
        k0 = r.integers(-50, 4_000, size=nd0).astype(np.int32) if dup else \
            r.permutation(5_000)[:nd0].astype(np.int32)
        k1 = r.integers(0, 3_000, size=nd1).astype(np.int32) if dup else \
            r.permutation(3_000)[:nd1].astype(np.int32)
        if nd1 > 2 and i % 3 == 0:
            k1[0] = -(2**31)  # the sentinel pattern as a real key
        pay1 = r.integers(-20, 20 + i, size=nd1).astype(np.int32)
        fk0 = r.integers(-60, 5_000, size=nf).astype(np.int32)
        fk1 = r.integers(-5, 3_000, size=nf).astype(np.int32)
        if nf > 10 and i % 3 == 0:
            fk1[:5] = -(2**31)
        g = r.integers(0, 40, size=nf).astype(np.int32)
        v = r.integers(-10**9, 10**9, size=nf).astype(np.int64)
        terms = [[], [(2, "lt", 30)], [(2, "range", 5, 35), (1, "ne", 7)]][i % 3]
        fact = [fk0, v, g, fk1]
        dims = [dict(fk=0, key=k0, payload=None), dict(fk=3, key=k1, payload=pay1)]
        specs.append((fact, terms, dims, key_sets[i % 4], agg_sets[(i // 2) % 4], 4_096))
    return specs


def test_batch_mixed_plans_of_one_shape():
    announce("batch mixed two-dim plans", 24)
    specs = mixed_specs(202, 24)
    b = run_batch(specs)
    for i, (spec, plan) in enumerate(zip(specs, b.plans)):
        assert_groups(plan.result(), oracle_of(spec), spec[4], f"mixed instance {i}")


def test_batch_int64_dims_and_no_dims():
    announce("batch int64 dims")
    r = np.random.default_rng(303)
    specs64, specs0 = [], []
    for i in range(6):
        n, nd = [10, 5_000, 70_001][i % 3], [1, 3_000][i % 2]
        key = r.integers(-2**62, 2**62, size=nd).astype(np.int64)
        key[::7] = np.iinfo(np.int64).min
        fk = np.where(r.random(n) < 0.7, r.choice(key, size=n), r.integers(-5, 5, size=n))
        g = r.integers(0, 30, size=n).astype(np.int32)
        v = r.integers(-10**6, 10**6, size=n).astype(np.int64)
        specs64.append(([fk.astype(np.int64), g, v], [], [dict(fk=0, key=key, payload=None)],
                        [("fact", 1)], [("sum", 2), ("count", None)], 64))
        specs0.append(([fk.astype(np.int64), g, v], [(1, "ge", 3)], [], [("fact", 1)] if i % 2 else [],
                       [("sum", 2), ("min", 2)], 64))
    for name, specs in (("int64 dims", specs64), ("no dims", specs0)):
        b = run_batch(specs)
        for i, (spec, plan) in enumerate(zip(specs, b.plans)):
            assert_groups(plan.result(), oracle_of(spec), spec[4], f"{name} instance {i}")


@pytest.mark.parametrize("chunk,grid", [(1, 0), (3, 7), (8, 0), (64, 1)])
def test_batch_work_split_does_not_change_results(chunk, grid):
    announce("batch work split", chunk, grid)
    insts = join_instances(404, 12, (100, 20_000), (1_000, 200_000), (8, 2_000))
    specs = [join_spec(i) for i in insts]
    b = run_batch(specs, t0=rel.tuning(chunk_tiles=chunk, grid=grid))
    for i, (spec, plan) in enumerate(zip(specs, b.plans)):
        assert_groups(plan.result(), oracle_of(spec), AGGS, f"chunk {chunk} grid {grid} inst {i}")


def test_batch_graph_replays():
    """The captured graph replayed several times, with eager work and
    synchronisations between replays, and after the inputs change in place:
    every replay equals the oracle on the inputs current at its launch."""
    announce("batch graph replays")
    insts = join_instances(505, 10, (100, 20_000), (1_000, 150_000), (8, 1_000))
    specs = [join_spec(i) for i in insts]
    plans = [device_plan(s) for s in specs]
    b = rel.PreparedBatch(plans)
    b.capture()
    want = [oracle_of(s) for s in specs]
    for rep in range(3):
        b.launch_graph()
        torch.cuda.synchronize()
        for i, plan in enumerate(b.plans):
            assert_groups(plan.result(), want[i], AGGS, f"replay {rep} instance {i}")
        # unrelated eager work between replays
        x = torch.arange(1 << 20, device="cuda", dtype=torch.int64)
        assert int(x.sum().item()) == (1 << 20) * ((1 << 20) - 1) // 2
    # change every probe value in place; the next replay reads the new values
    for plan, spec in zip(plans, specs):
        plan._keep[0][1].add_(3)
        spec[0][1] = spec[0][1] + 3
    b.launch_graph()
    torch.cuda.synchronize()
    for i, (plan, spec) in enumerate(zip(b.plans, specs)):
        assert_groups(plan.result(), oracle_of(spec), AGGS, f"replay after update, instance {i}")
    # the eager path on the same batch agrees as well
    b.launch()
    torch.cuda.synchronize()
    for i, (plan, spec) in enumerate(zip(b.plans, specs)):
        assert_groups(plan.result(), oracle_of(spec), AGGS, f"eager after graph, instance {i}")
    b.release()


def test_batch_plans_sharing_one_fact_table():
    """Plans over the same resident fact columns (their tile ranges are
    interleaved across plans): different date ranges, dims and group
    attributes, each equal to the oracle."""
    announce("batch shared fact table")
    d = datagen.star_schema(seed=17, n_fact=250_001, n_dim_a=20_000, n_dim_b=1_000)
    r = np.random.default_rng(606)
    city = (r.permutation(1_000) % 200).astype(np.int32)
    segment = (r.permutation(20_000) % 5_000).astype(np.int32)
    fact = [d["fk_a"], d["fk_b"], d["date"], d["price"], d["flag"]]
    dfact = [dev(c) for c in fact]
    attrs = [(1, d["dim_b_key"], d["dim_b_region"]), (1, d["dim_b_key"], city),
             (0, d["dim_a_key"], segment)]
    ddims = {k: dev(a) for k, a in [("a", d["dim_a_key"]), ("b", d["dim_b_key"]),
                                     ("region", d["dim_b_region"]), ("city", city),
                                     ("segment", segment)]}
    dev_attr = [(1, ddims["b"], ddims["region"]), (1, ddims["b"], ddims["city"]),
                (0, ddims["a"], ddims["segment"])]
    aggs = [("sum", 3), ("count", None)]
    specs, plans = [], []
    for q in range(9):
        w = int(r.integers(25, 1_300))
        lo = int(r.integers(0, 2_557 - w))
        a = q % 3
        fk, key, pay = attrs[a]
        terms = [(2, "range", lo, lo + w)]
        specs.append((fact, terms, [dict(fk=fk, key=key, payload=pay)], [("dim", 0)], aggs, 5_000))
        fk_d, key_d, pay_d = dev_attr[a]
        plans.append(rel.Plan(dfact, terms, [dict(fk=fk_d, key=key_d, payload=pay_d)],
                              [("dim", 0)], aggs, 5_000))
    b = rel.PreparedBatch(plans)
    b.launch()
    torch.cuda.synchronize()
    for q, (spec, plan) in enumerate(zip(specs, b.plans)):
        assert_groups(plan.result(), oracle_of(spec), aggs, f"shared-scan query {q}")


def test_autotuner_candidates_agree_and_records_apply_to_batches():
    """Every tuning candidate returns the same groups (the tuner raises
    otherwise: a race detector), and a batch whose instances carry the tuned
    records still equals the oracle."""
    import json

    from paper_2508_04701_amd import autotune
    announce("autotuner")
    insts = join_instances(707, 6, (1_000, 20_000), (10_000, 300_000), (8, 5_000))
    specs = [join_spec(i) for i in insts]
    cache = autotune.Cache()
    tunings = []
    for spec in specs:
        fact, terms, dims, keys, aggs, mg = spec
        dfact = [dev(c) for c in fact]
        ddims = [dict(fk=0, key=dev(dims[0]["key"]), payload=dev(dims[0]["payload"]))]
        rec = autotune.tune_plan(
            lambda t: rel.PreparedPipeline(dfact, terms, ddims, keys, aggs, mg, t))
        assert set(rec["candidates"]) == {json.dumps(c, sort_keys=True)
                                          for c in autotune.CANDIDATES}
        b = autotune.plan_bucket(len(fact[0]), [len(dims[0]["key"])], mg)
        cache.put(autotune.cache_key("join_groupby", b), rec)
        tunings.append(autotune.tuning_for(cache, "join_groupby", len(fact[0]),
                                           [len(dims[0]["key"])], mg))
    plans = [device_plan(s, t) for s, t in zip(specs, tunings)]
    b = rel.PreparedBatch(plans)
    b.launch()
    torch.cuda.synchronize()
    for i, (spec, plan) in enumerate(zip(specs, b.plans)):
        assert_groups(plan.result(), oracle_of(spec), AGGS, f"tuned instance {i}")


def test_autotuner_groupby_fanout_candidates_agree():
    """The group-by tuner's candidates (single pass, automatic and forced
    partition fan-outs, no first-scatter LDS table) return the same groups,
    and the kept record reproduces the oracle."""
    from paper_2508_04701_amd import autotune
    announce("autotuner group-by")
    r = np.random.default_rng(808)
    n = 1_000_003
    k = r.integers(0, 200_000, size=n).astype(np.int64)
    v = r.integers(-10**9, 10**9, size=n).astype(np.int64)
    aggs = [("sum", 0), ("count", None), ("min", 0), ("max", 0)]
    rec = autotune.tune_groupby([dev(k)], [dev(v)], aggs, 200_000)
    assert len(rec["candidates"]) == len(autotune.GROUPBY_CANDIDATES)
    got = rel.groupby_agg([dev(k)], [dev(v)], aggs, max_groups=200_000,
                          t=autotune.to_tuning(rec["tuning"]))
    assert_groups(got, oracle.groupby([k], [v], aggs), aggs, "tuned group-by")


def test_native_autotuner_records_and_lookups(tmp_path):
    """rel_autotune through the C-ABI: every candidate (load factor, fan-out,
    block shape, LDS group table, replicas, record partitions) returns the
    same groups (it fails otherwise), one record per bucket lands in the
    JSON cache with all eighteen candidates timed, rel_autotune_lookup
    returns it, and a batch whose instances carry the looked-up records
    equals the oracle."""
    import json

    from paper_2508_04701_amd import autotune
    announce("native autotuner")
    insts = join_instances(717, 4, (1_000, 200_000), (10_000, 2_000_000), (8, 20_000))
    specs = [join_spec(i) for i in insts]
    path = str(tmp_path / "tune.json")
    plans = [device_plan(s) for s in specs]
    autotune.tune_batch_plans(plans, path)
    recs = json.load(open(path))
    keys = {k for k in recs if "/pipeline_batch/" in k}
    assert len(keys) == len({autotune.plan_bucket(len(s[0][0]), [len(s[2][0]["key"])], s[5])
                             for s in specs})
    for k in keys:
        assert len(recs[k]["candidates"]) == 18 and recs[k]["ms"] > 0
    tuned = [device_plan(s, autotune.lookup(path, p)) for s, p in zip(specs, plans)]
    assert all(autotune.lookup(path, p) is not None for p in plans)
    b = rel.PreparedBatch(tuned)
    b.launch()
    torch.cuda.synchronize()
    for i, (spec, plan) in enumerate(zip(specs, b.plans)):
        assert_groups(plan.result(), oracle_of(spec), AGGS, f"native-tuned instance {i}")


def test_batch_direct_tables_built_in_slices_and_parts():
    """Dims large enough that the direct-table build spreads over many LDS
    workgroups: with payloads, windows of 16k keys (the rows grouped by
    window first); membership only, slices of the key range split over parts
    of the build rows. Unique keys (a direct table), and the same keys with
    one key repeated in another part (the duplicate must be seen, so the dim
    falls back to its hash table and the repeated key's rows are counted
    twice)."""
    announce("batch direct slices")
    r = np.random.default_rng(77)
    nb = 1_300_000  # three parts of the build rows; two slices of bits
    # keys with gaps in their range, so that probes read the bitmap
    keys = (r.choice(1_800_000, size=nb, replace=False) + 5).astype(np.int32)
    grp = r.integers(0, 40, size=nb).astype(np.int32)
    dup_keys = keys.copy()
    dup_keys[1_200_000] = dup_keys[10]  # rows in the first and the last part
    npr = 600_000
    pk = r.integers(0, 1_800_010, size=npr).astype(np.int32)
    pv = r.integers(-1000, 1000, size=npr).astype(np.int64)
    specs = []
    for k in (keys, dup_keys):
        specs.append(([pk, pv], [], [dict(fk=0, key=k, payload=grp)], [("dim", 0)], AGGS, 64))
    b = run_batch(specs)
    for i, (spec, plan) in enumerate(zip(specs, b.plans)):
        assert_groups(plan.result(), oracle_of(spec), AGGS, f"instance {i}")
    # membership-only dims: slices and parts
    aggs = [("count", None), ("sum", 1), ("min", 1)]
    specs = [([pk, pv], [], [dict(fk=0, key=k, payload=None)], [], aggs, 1)
             for k in (keys, dup_keys)]
    b = run_batch(specs)
    for i, (spec, plan) in enumerate(zip(specs, b.plans)):
        assert_groups(plan.result(), oracle_of(spec), aggs, f"membership instance {i}")


def record_specs(seed):
    """Join + group-by plans whose groups outgrow the fused pass's LDS table,
    so that their spilled rows go through the record passes: uniform groups
    from 3k to 600k, Zipf-skewed groups, records of one, two and three words
    (COUNT only; one value column; two value columns), a plan with three
    value columns (no records: its spilled rows use atomics), a plan whose
    probes all miss, one with no probe rows, two int8 group keys (a dim
    attribute and a fact column, negative values included) whose packed key
    takes 16 bits, and 600k groups over 1024 partitions."""
    r = np.random.default_rng(seed)
    specs = []

    def plan(n_build, n_probe, groups, aggs, grp=None, miss=False, ncols=1, int8_keys=False):
        keys = r.permutation(n_build).astype(np.int32)
        if grp is None:
            grp = r.integers(0, groups, size=n_build).astype(np.int32)
        lo = n_build + 10 if miss else 0
        pk = r.integers(lo, lo + int(n_build * 1.1) + 1, size=n_probe).astype(np.int32)
        vals = [r.integers(-10**6, 10**6, size=n_probe).astype(np.int64) for _ in range(ncols)]
        group_keys = [("dim", 0)]
        fact = [pk] + vals
        if int8_keys:
            grp = r.integers(-128, 128, size=n_build).astype(np.int8)
            fact.append(r.integers(-128, 128, size=n_probe).astype(np.int8))
            group_keys = [("dim", 0), ("fact", len(fact) - 1)]
        specs.append((fact, [], [dict(fk=0, key=keys, payload=grp)], group_keys, aggs,
                      max(1, groups)))

    plan(200_000, 300_000, 3_000, AGGS)
    plan(400_000, 500_001, 40_000, AGGS)
    plan(600_000, 700_000, 150_000, [("sum", 1), ("count", None)])
    plan(1_000_000, 1_200_000, 600_000, [("sum", 1), ("count", None)])  # 1024 partitions
    zipf = (datagen.zipf_ranks(seed, 9, 60_000, 1.1, 300_000) - 1).astype(np.int32)
    plan(300_000, 400_000, 60_000, AGGS, grp=zipf)
    plan(100_000, 200_000, 20_000, [("count", None)])
    plan(100_000, 250_000, 30_000, [("sum", 1), ("max", 2), ("avg", 2)], ncols=2)
    plan(100_000, 150_000, 30_000, [("sum", 1), ("min", 2), ("max", 3)], ncols=3)
    plan(50_000, 100_000, 10_000, AGGS, miss=True)
    plan(50_000, 0, 10_000, AGGS)
    plan(200_000, 400_000, 65_536, AGGS, int8_keys=True)
    return specs


def run_tuned(specs, tunings):
    b = rel.PreparedBatch([device_plan(s, t) for s, t in zip(specs, tunings)])
    b.launch()
    torch.cuda.synchronize()
    return b


@pytest.mark.parametrize("fanout", [0, 4, 1024, -1])
def test_batch_spilled_rows_as_records(fanout):
    """Rows that find no LDS group slot become records, grouped by partition
    and folded per partition in LDS (fanout 0: partitions sized for the
    aggregation table; 4: far fewer, so most keys of a partition miss its
    LDS table and update the global table directly; 1024: the most, several
    per scatter thread; -1: no records, device atomics): every plan equals
    the oracle."""
    announce("batch records", fanout)
    specs = record_specs(1212)
    t = rel.tuning(fanout=fanout)
    b = run_tuned(specs, [t] * len(specs))
    for i, (spec, plan) in enumerate(zip(specs, b.plans)):
        assert_groups(plan.result(), oracle_of(spec), spec[4], f"fanout {fanout} plan {i}")


def test_batch_records_graph_replays():
    """The record passes inside a captured graph: their counters and piece
    list start from zero on every replay."""
    announce("batch records graph")
    specs = record_specs(1313)[:4]
    b = rel.PreparedBatch([device_plan(s) for s in specs])
    b.capture()
    want = [oracle_of(s) for s in specs]
    for rep in range(3):
        b.launch_graph()
        torch.cuda.synchronize()
        for i, plan in enumerate(b.plans):
            assert_groups(plan.result(), want[i], specs[i][4], f"replay {rep} plan {i}")
        x = torch.arange(1 << 20, device="cuda", dtype=torch.int64)
        assert int(x.sum().item()) == (1 << 20) * ((1 << 20) - 1) // 2
    b.release()


def test_batch_records_beside_an_lds_table():
    """A tuning that keeps an LDS group table (1024 slots) for plans with
    records: rows whose groups hold an LDS slot are flushed from it, the
    others become records, and both reach the one global table. Uniform and
    Zipf-skewed groups (the hot ones stay in LDS)."""
    announce("batch records with an LDS table")
    specs = record_specs(1414)[:4]
    t = rel.tuning(lds_slots=1024)
    b = run_tuned(specs, [t] * len(specs))
    for i, (spec, plan) in enumerate(zip(specs, b.plans)):
        assert_groups(plan.result(), oracle_of(spec), spec[4], f"plan {i}")
