"""Out-of-core execution (rel_pipeline_stream): the fused plan over fact
columns in pinned host memory, streamed through two device staging slots in
chunks while the previous chunk is aggregated, against the oracle on the
whole table - ragged last chunks, a single chunk, an empty table, duplicate
dim keys (the per-chunk enumeration pass), hash-table and direct-table dims,
and repeated launches."""

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import announce, assert_groups, canon_groups, dev
from paper_2508_04701_amd import datagen, rel

pytestmark = pytest.mark.gpu

STAR_AGGS = [("sum", 3), ("count", None), ("avg", 3), ("min", 3), ("max", 3)]


def pinned(a):
    return torch.from_numpy(np.ascontiguousarray(a)).pin_memory()


def star(n, seed=51):
    d = datagen.star_schema(seed=seed, n_fact=n, n_dim_a=20_000, n_dim_b=2_000)
    fact = [d["fk_a"], d["fk_b"], d["date"], d["price"], d["flag"]]
    dims = [dict(fk=0, key=d["dim_a_key"], payload=None),
            dict(fk=1, key=d["dim_b_key"], payload=d["dim_b_region"])]
    return fact, dims


def run(fact, dims, terms, keys, aggs, chunk, t=None, max_groups=128, launches=1):
    ddims = [dict(fk=x["fk"], key=dev(x["key"]),
                  payload=None if x.get("payload") is None else dev(x["payload"])) for x in dims]
    plan = rel.StreamedPipeline([pinned(c) for c in fact], terms, ddims, keys, aggs, max_groups,
                                chunk, t)
    out = []
    for _ in range(launches):
        plan.launch()
        out.append(plan.result())
    return out


@pytest.mark.parametrize("n,chunk", [(0, 2048), (5, 2048), (2048, 2048), (300_001, 2048 * 7),
                                     (1_000_000, 2048 * 100)])
@pytest.mark.parametrize("direct", [False, True])
def test_streamed_star_schema(n, chunk, direct):
    announce("out-of-core star", n, chunk, direct)
    fact, dims = star(n)
    t = None if direct else rel.tuning(flags=rel.TUNE_NO_DIRECT)
    terms, keys = [(2, "lt", 767)], [("dim", 1), ("fact", 4)]
    got = run(fact, dims, terms, keys, STAR_AGGS, chunk, t, launches=2)
    want = oracle.pipeline(fact, terms, dims, keys, STAR_AGGS)
    for g in got:
        assert_groups(g, want, STAR_AGGS, f"streamed n={n} chunk={chunk} direct={direct}")


def test_streamed_duplicate_dim_keys():
    announce("out-of-core dup dims")
    fact, dims = star(200_000, seed=52)
    kb = dims[1]["key"].copy()
    kb[:100] = kb[100:200]  # every chunk meets duplicate keys
    dims[1]["key"] = kb
    terms, keys = [(2, "range", 100, 1500)], [("dim", 1), ("fact", 4)]
    got = run(fact, dims, terms, keys, STAR_AGGS, 2048 * 5)[0]
    assert_groups(got, oracle.pipeline(fact, terms, dims, keys, STAR_AGGS), STAR_AGGS, "dup dims")


def test_streamed_equals_resident():
    announce("out-of-core vs resident")
    fact, dims = star(500_000, seed=53)
    terms, keys = [(2, "ge", 1000)], [("dim", 1)]
    aggs = [("sum", 3), ("count", None)]
    streamed = run(fact, dims, terms, keys, aggs, 2048 * 16)[0]
    ddims = [dict(fk=x["fk"], key=dev(x["key"]),
                  payload=None if x.get("payload") is None else dev(x["payload"])) for x in dims]
    resident = rel.pipeline([dev(c) for c in fact], terms, ddims, keys, aggs, 128)
    a, b = canon_groups(*streamed), canon_groups(*resident)
    assert all(np.array_equal(x, y) for x, y in zip(a[0] + a[1], b[0] + b[1]))
