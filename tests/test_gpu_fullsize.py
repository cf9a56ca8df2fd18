"""GPU parity at the benchmark's full sizes, in the configurations bench.py
times: the 600M-row star schema through rel_pipeline against the oracle on
all rows (≈1 minute of single-threaded oracle time), and the 256-instance
batch (1.55G probe rows) through rel_pipeline_batch against 256 single
rel_pipeline calls, with the oracle on the smallest instances."""

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import announce, assert_groups, canon_groups
from paper_2508_04701_amd import datagen, rel

pytestmark = pytest.mark.gpu

STAR_AGGS = [("sum", 3), ("count", None), ("avg", 3), ("min", 3), ("max", 3)]


def test_star_schema_600m_rows_against_oracle():
    """The benchmark's plan with both dims in hash tables (the headline
    configuration) and with direct tables, each launched twice, against one
    oracle run over all 600M rows."""
    announce("full-size star schema 600M")
    d = datagen.star_schema(seed=datagen.SEED0 + 2, n_fact=600_000_000)
    fact = [d["fk_a"], d["fk_b"], d["date"], d["price"], d["flag"]]
    dims = [dict(fk=0, key=d["dim_a_key"], payload=None),
            dict(fk=1, key=d["dim_b_key"], payload=d["dim_b_region"])]
    keys = [("dim", 1), ("fact", 4)]
    terms = [(2, "lt", 767)]
    dev = [torch.from_numpy(c).cuda() for c in fact]
    ddims = [dict(fk=0, key=torch.from_numpy(d["dim_a_key"]).cuda(), payload=None),
             dict(fk=1, key=torch.from_numpy(d["dim_b_key"]).cuda(),
                  payload=torch.from_numpy(d["dim_b_region"]).cuda())]
    results = {}
    for name, t in (("hash tables", rel.tuning(flags=rel.TUNE_NO_DIRECT)), ("direct tables", None)):
        announce("full-size star schema 600M,", name)
        plan = rel.PreparedPipeline(dev, terms, ddims, keys, STAR_AGGS, max_groups=128, t=t)
        plan.launch()
        got = plan.result()
        # the same launch again: results must not depend on the run
        plan.launch()
        again = plan.result()
        a, b = canon_groups(*got), canon_groups(*again)
        assert all(np.array_equal(x, y) for x, y in zip(a[0] + a[1], b[0] + b[1])), name
        results[name] = got
        del plan
    del dev, ddims
    torch.cuda.empty_cache()
    want = oracle.pipeline(fact, terms, dims, keys, STAR_AGGS)
    assert len(want[1][0]) == 75
    for name, got in results.items():
        assert_groups(got, want, STAR_AGGS, f"star schema 600M, {name}")


def test_batch_256_instances_full_size():
    announce("full-size batch 256 instances")
    seed = datagen.SEED0 + 4
    shapes = datagen.batch_shapes(seed=seed)
    aggs = [("sum", 1), ("count", None)]
    singles, plans, host = [], [], []
    for i, s in enumerate(shapes):
        d = datagen.batch_instance(seed, i, **s)
        fact = [torch.from_numpy(d["probe_key"]).cuda(), torch.from_numpy(d["probe_val"]).cuda()]
        dims = [dict(fk=0, key=torch.from_numpy(d["build_key"]).cuda(),
                     payload=torch.from_numpy(d["build_grp"]).cuda())]
        g = max(1, s["n_groups"])
        singles.append(rel.PreparedPipeline(fact, [], dims, [("dim", 0)], aggs, g))
        plans.append(rel.Plan(fact, [], dims, [("dim", 0)], aggs, g))
        host.append((s, d))
    batch = rel.PreparedBatch(plans)
    for p in singles:
        p.launch()
    batch.launch()
    torch.cuda.synchronize()
    # the oracle on a stratified sample: the eight largest instances (their
    # groups spill from the LDS tables into replicated global tables), the
    # small ones, and every 16th of the rest
    by_size = sorted(range(len(shapes)), key=lambda i: shapes[i]["n_probe"])
    sample = set(by_size[-8:]) | {i for i in by_size if shapes[i]["n_probe"] < 200_000} | \
        set(by_size[::16])
    checked = 0
    for i, (single, plan) in enumerate(zip(singles, plans)):
        a, b = canon_groups(*single.result()), canon_groups(*plan.result())
        assert len(a[1][0]) == len(b[1][0]), f"instance {i}: group counts differ"
        assert all(np.array_equal(x, y) for x, y in zip(a[0] + a[1], b[0] + b[1])), \
            f"instance {i}: batched differs from the single call"
        if i in sample:
            s, d = host[i]
            want = oracle.pipeline([d["probe_key"], d["probe_val"]], [],
                                   [dict(fk=0, key=d["build_key"], payload=d["build_grp"])],
                                   [("dim", 0)], aggs)
            assert_groups(plan.result(), want, aggs, f"instance {i} vs oracle")
            checked += 1
    assert checked >= 8 + 16


def test_skewed_join_and_groupby_full_size_properties():
    """100M unique int64 build keys, 400M Zipf(1) probes, ~10M groups: the
    oracle would take many minutes here, so the checks are properties that
    hold at any size, computed with plain torch reductions: every probe row
    appears in exactly one pair whose keys are equal; COUNT sums to the row
    count and SUM to the column's exact total; the group count equals the
    number of distinct keys; and every group's COUNT/SUM/MIN/MAX/AVG equals
    a sort-and-segment reduction of the same column."""
    announce("full-size skewed join + group-by")
    sk = datagen.skewed()
    bk = torch.from_numpy(sk["build_key"]).cuda()
    pk = torch.from_numpy(sk["probe_key"]).cuda()
    g = torch.from_numpy(sk["probe_grp"]).cuda()
    v = torch.from_numpy(sk["probe_val"]).cuda()
    del sk
    n = pk.numel()
    ob, op = rel.hash_join(bk, pk, out_cap=n)
    assert ob.numel() == n
    seen = torch.zeros(n, dtype=torch.int32, device="cuda")
    seen.index_add_(0, op.long(), torch.ones(n, dtype=torch.int32, device="cuda"))
    assert bool((seen == 1).all()), "every probe row must match exactly once"
    assert torch.equal(bk[ob.long()], pk[op.long()]), "paired keys must be equal"
    del ob, op, seen
    aggs = [("sum", 0), ("count", None), ("avg", 0), ("min", 0), ("max", 0)]
    keys, vals = rel.groupby_agg([g], [v], aggs, max_groups=10_000_000)
    uniq, counts = torch.unique(g, return_counts=True)
    assert keys[0].numel() == uniq.numel()
    assert int(vals[1].sum()) == n
    assert int(vals[0].sum()) == int(v.sum())
    order = torch.argsort(keys[0])
    k_sorted = keys[0][order]
    assert torch.equal(k_sorted, uniq)
    assert torch.equal(vals[1][order], counts)
    # every group against an independent sort-and-segment reduction (torch's
    # unique + scatter_reduce on int64): SUM, COUNT, MIN, MAX exactly, AVG as
    # the binary64 quotient of the exact SUM and COUNT
    _, inv = torch.unique(g, return_inverse=True)
    nu = uniq.numel()
    ssum = torch.zeros(nu, dtype=torch.int64, device="cuda").scatter_add_(0, inv, v)
    smin = torch.full((nu,), 2**63 - 1, dtype=torch.int64, device="cuda").scatter_reduce_(
        0, inv, v, reduce="amin")
    smax = torch.full((nu,), -(2**63), dtype=torch.int64, device="cuda").scatter_reduce_(
        0, inv, v, reduce="amax")
    del inv
    assert torch.equal(vals[0][order], ssum), "SUM of every group"
    assert torch.equal(vals[3][order], smin), "MIN of every group"
    assert torch.equal(vals[4][order], smax), "MAX of every group"
    # SUM < 2^53 here, so the double conversions are exact and the quotient is
    # one correctly rounded division
    assert int(ssum.max()) < 2**53
    assert torch.equal(vals[2][order], ssum.double() / counts.double()), "AVG of every group"
