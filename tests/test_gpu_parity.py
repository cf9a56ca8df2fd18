"""GPU parity: every entry point of the C-ABI against the oracle on the same
seeded inputs. Filter output must match exactly (ascending row ids); join
pairs and groups must match exactly after canonical sorting, AVG bit for
bit (tolerance 0)."""

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import announce, assert_groups, assert_pairs, dev, rowids
from paper_2508_04701_amd import datagen, rel

pytestmark = pytest.mark.gpu

I32_MIN, I32_MAX = -(2**31), 2**31 - 1
I64_MIN, I64_MAX = -(2**63), 2**63 - 1


def rng(seed):
    return np.random.default_rng(seed)


def col_with_extremes(r, n, dtype, lo, hi, frac=0.05):
    v = r.integers(lo, hi, size=n).astype(dtype)
    info = np.iinfo(dtype)
    pick = r.random(n) < frac
    v[pick] = r.choice(np.array([info.min, info.max, -1, 0], dtype=dtype), size=int(pick.sum()))
    return v


# ------------------------------------------------------------------ filter

@pytest.mark.parametrize("n", [0, 1, 7, 4095, 4097, 8191, 8192, 8193, 100_003, 1_000_000])
def test_filter_sizes(n):
    announce("filter sizes", n)
    r = rng(n)
    date = r.integers(0, 2557, size=n).astype(np.int32)
    got = rel.filter([dev(date)], [(0, "lt", 767)])
    want = oracle.filter([date], [(0, "lt", 767)])
    assert np.array_equal(rowids(got), want)


@pytest.mark.parametrize("seed", range(8))
def test_filter_mixed_terms(seed):
    r = rng(100 + seed)
    n = int(r.integers(20_000, 120_000))
    cols = [col_with_extremes(r, n, np.int8, -20, 20), col_with_extremes(r, n, np.int32, -50, 50),
            col_with_extremes(r, n, np.int64, -10**6, 10**6)]
    ops = list(rel.CMP)
    terms = []
    for _ in range(int(r.integers(1, 5))):
        c = int(r.integers(0, 3))
        op = ops[int(r.integers(0, len(ops)))]
        scale = [20, 50, 10**6][c]
        lo = int(r.integers(-scale, scale))
        terms.append((c, op, lo, lo + int(r.integers(0, scale))))
    announce("filter mixed", seed, n, terms)
    # unaligned views exercise the scalar load path
    offset = seed % 2
    dcols = [dev(c) for c in cols] if not offset else [dev(np.concatenate([c[:1], c]))[1:] for c in cols]
    got = rel.filter(dcols, terms)
    want = oracle.filter(cols, terms)
    assert np.array_equal(rowids(got), want)


def test_filter_selection_vectors():
    r = rng(7)
    n = 300_000
    x = r.integers(-100, 100, size=n).astype(np.int64)
    y = r.integers(0, 10, size=n).astype(np.int32)
    terms = [(0, "range", -30, 40), (1, "ne", 3)]
    for name, sel in (("sorted", np.sort(r.choice(n, size=n // 3, replace=False))),
                      ("shuffled", r.permutation(n)[: n // 2]),
                      ("empty", np.zeros(0, np.int64))):
        announce("filter selection", name)
        sel = sel.astype(np.uint32)
        got = rel.filter([dev(x), dev(y)], terms, idx=dev(sel.view(np.int32)))
        want = oracle.filter([x, y], terms, sel=sel)
        assert np.array_equal(rowids(got), want), name


@pytest.mark.parametrize("n", [64 * 16384, 64 * 16384 + 1, 3_000_017])
def test_filter_across_offset_groups(n):
    """Sizes at and past one group of 64 tiles (16384 rows each), whose
    offsets the scan pass sums per group: ids must stay ascending and exact
    across group boundaries, with a ragged last tile; two int32 terms (the
    int32-only mark kernel) and an int64 term (the general one)."""
    announce("filter offset groups", n)
    r = rng(n % 1000)
    a = r.integers(0, 1000, size=n).astype(np.int32)
    b = r.integers(-50, 50, size=n).astype(np.int32)
    c = r.integers(-(10**12), 10**12, size=n).astype(np.int64)
    for cols, terms in (([a, b], [(0, "lt", 300), (1, "ge", -10)]),
                        ([a, c], [(0, "range", 100, 900), (1, "lt", 0)])):
        got = rel.filter([dev(x) for x in cols], terms)
        want = oracle.filter(cols, terms)
        assert np.array_equal(rowids(got), want), terms
    # through a selection vector longer than one group of tiles
    sel = r.permutation(n)[: n * 2 // 3].astype(np.uint32)
    got = rel.filter([dev(a), dev(b)], [(0, "lt", 500)], idx=dev(sel.view(np.int32)))
    want = oracle.filter([a, b], [(0, "lt", 500)], sel=sel)
    assert np.array_equal(rowids(got), want), "selection vector"


def test_filter_output_capacity():
    announce("filter capacity")
    r = rng(9)
    n = 50_000
    x = r.integers(0, 100, size=n).astype(np.int32)
    want = oracle.filter([x], [(0, "lt", 50)])
    out = torch.full((1000,), -7, dtype=torch.int32, device="cuda")
    d_count = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = rel.workspace(rel.filter_ws(n))
    rel.filter_async([dev(x)], [(0, "lt", 50)], out, d_count, ws)
    assert int(d_count.item()) == len(want)
    assert np.array_equal(rowids(out), want[:1000])


def test_filter_all_and_nothing():
    x = np.arange(-5000, 5000, dtype=np.int64)
    announce("filter all/nothing")
    every = rel.filter([dev(x)], [(0, "range", I64_MIN, I64_MAX)])
    assert np.array_equal(rowids(every), np.arange(10_000, dtype=np.uint32))
    assert rel.filter([dev(x)], [(0, "gt", I64_MAX)]).numel() == 0


# --------------------------------------------------------------- hash join

def join_case(case, dtype, r):
    info = np.iinfo(dtype)
    if case == "unique":
        b = r.permutation(20_000).astype(dtype) * 7 - 3
        p = r.integers(-10, 160_000, size=90_000).astype(dtype)
    elif case == "unique_sentinel":
        # unique build keys, one of them the sentinel pattern: the probe ends
        # every walk at its first match, out-of-band keys included
        b = r.permutation(20_000).astype(dtype) * 7 - 3
        b[123] = info.min
        p = r.integers(-10, 160_000, size=90_001).astype(dtype)
        p[r.random(p.size) < 0.01] = info.min
    elif case == "dups":
        b = r.integers(0, 3000, size=12_000).astype(dtype)
        p = r.integers(0, 4000, size=30_000).astype(dtype)
    elif case == "sentinel":
        b = r.choice(np.array([info.min, info.max, -1, 0, 5], dtype=dtype), size=300)
        p = r.choice(np.array([info.min, info.max, -1, 0, 7], dtype=dtype), size=500)
    elif case == "empty_build":
        b = np.zeros(0, dtype)
        p = r.integers(0, 10, size=1000).astype(dtype)
    else:
        b = r.integers(0, 10, size=1000).astype(dtype)
        p = np.zeros(0, dtype)
    return b, p


@pytest.mark.parametrize("dtype", [np.int32, np.int64], ids=["i32", "i64"])
@pytest.mark.parametrize("case", ["unique", "unique_sentinel", "dups", "sentinel", "empty_build",
                                  "empty_probe"])
def test_hash_join(case, dtype):
    announce("join", case, np.dtype(dtype).name)
    seed = {"unique": 1, "unique_sentinel": 6, "dups": 2, "sentinel": 3, "empty_build": 4,
            "empty_probe": 5}[case]
    b, p = join_case(case, dtype, rng(seed))
    got = rel.hash_join(dev(b), dev(p))
    assert_pairs(got, oracle.hash_join(b, p), case)


def partitioned_build_case(case, dtype, r):
    """Build sides of at least 4 LDS ranges (32768 int32 / 16384 int64 keys
    and more), with runs that cross range ends."""
    info = np.iinfo(dtype)
    if case == "unique":
        b = r.permutation(70_000).astype(dtype) * 3 - 7
        p = r.integers(-100, 215_000, size=200_001).astype(dtype)
    elif case == "dups":
        # ~23 copies per key: long runs, spills past range ends
        b = r.integers(0, 3000, size=70_000).astype(dtype)
        p = r.integers(0, 3500, size=20_000).astype(dtype)
    elif case == "sentinel":
        b = r.integers(-50_000, 50_000, size=70_000).astype(dtype)
        b[r.random(b.size) < 0.05] = info.min
        p = r.integers(-60_000, 60_000, size=50_000).astype(dtype)
        p[r.random(p.size) < 0.05] = info.min
    else:  # one key repeated 6000 times among unique keys
        b = r.permutation(70_000).astype(dtype)
        b[r.choice(b.size, 6000, replace=False)] = 12345
        p = r.integers(0, 80_000, size=100_000).astype(dtype)
    return b, p


@pytest.mark.parametrize("dtype", [np.int32, np.int64], ids=["i32", "i64"])
@pytest.mark.parametrize("case", ["unique", "dups", "sentinel", "hot"])
@pytest.mark.parametrize("fanout", [4, 16384])
def test_hash_join_partitioned_build(case, dtype, fanout):
    """The partitioned build (ranges of the slot array built in LDS, runs past
    a range end inserted afterwards), forced by the fan-out: 4 partitions of
    several ranges each, or one partition per range."""
    announce("join partitioned build", case, np.dtype(dtype).name, fanout)
    seed = {"unique": 11, "dups": 12, "sentinel": 13, "hot": 14}[case]
    b, p = partitioned_build_case(case, dtype, rng(seed))
    t = rel.tuning(fanout=fanout)
    single = rel.hash_join_ws(torch.from_numpy(b).dtype, b.size, rel.tuning(fanout=-1))
    assert rel.hash_join_ws(torch.from_numpy(b).dtype, b.size, t) >= single + 32 * b.size
    got = rel.hash_join(dev(b), dev(p), t=t)
    assert_pairs(got, oracle.hash_join(b, p), f"partitioned {case}")


def test_hash_join_partitioned_build_with_row_ids():
    announce("join partitioned build idx")
    r = rng(15)
    b = r.integers(0, 40_000, size=90_000).astype(np.int64)
    p = r.integers(0, 45_000, size=60_000).astype(np.int64)
    bsel = np.sort(r.choice(90_000, size=50_000, replace=False)).astype(np.uint32)
    got = rel.hash_join(dev(b), dev(p), build_idx=dev(bsel.view(np.int32)),
                        t=rel.tuning(fanout=8))
    wb, wp = oracle.hash_join(b[bsel], p)
    wb2 = bsel[wb]
    order = np.lexsort((wb2, wp))
    assert_pairs(got, (wb2[order], wp[order]), "partitioned idx")


def test_hash_join_with_row_ids():
    announce("join with idx")
    r = rng(3)
    b = r.integers(0, 5000, size=8000).astype(np.int64)
    p = r.integers(0, 6000, size=40_000).astype(np.int64)
    bsel = np.sort(r.choice(8000, size=3000, replace=False)).astype(np.uint32)
    psel = r.permutation(40_000)[:25_000].astype(np.uint32)
    got = rel.hash_join(dev(b), dev(p), build_idx=dev(bsel.view(np.int32)),
                        probe_idx=dev(psel.view(np.int32)))
    wb, wp = oracle.hash_join(b[bsel], p[psel])
    wb2, wp2 = bsel[wb], psel[wp]     # row ids are original positions
    order = np.lexsort((wb2, wp2))
    assert_pairs(got, (wb2[order], wp2[order]), "idx")


def test_hash_join_capacity():
    announce("join capacity")
    r = rng(4)
    b = r.integers(0, 100, size=2000).astype(np.int32)
    p = r.integers(0, 100, size=2000).astype(np.int32)
    wb, wp = oracle.hash_join(b, p)
    ws = rel.workspace(rel.hash_join_ws(torch.int32, 2000))
    ob = torch.empty(100, dtype=torch.int32, device="cuda")
    op = torch.empty(100, dtype=torch.int32, device="cuda")
    d = torch.zeros(1, dtype=torch.int64, device="cuda")
    rel.hash_join_async(dev(b), dev(p), ob, op, d, ws)
    assert int(d.item()) == len(wb)
    # every written pair is a true match
    gb, gp = rowids(ob), rowids(op)
    assert np.array_equal(b[gb], p[gp])


# ---------------------------------------------------------------- group-by

ALL_AGGS = [("sum", 0), ("count", None), ("min", 0), ("max", 0), ("avg", 0), ("sum", 1),
            ("avg", 1), ("min", 2)]


def groupby_inputs(r, n, key_dtypes, ngroups):
    keys = []
    for dt in key_dtypes:
        hi = min(ngroups, np.iinfo(dt).max)
        keys.append(r.integers(-hi // 2, hi - hi // 2, size=n).astype(dt))
    vals = [col_with_extremes(r, n, np.int64, -10**12, 10**12, 0.01),
            r.integers(-1000, 1000, size=n).astype(np.int32),
            r.integers(-100, 100, size=n).astype(np.int8)]
    return keys, vals


@pytest.mark.parametrize("key_dtypes", [[], [np.int32], [np.int64], [np.int8, np.int32],
                                        [np.int32, np.int32], [np.int32, np.int8]],
                         ids=["none", "i32", "i64", "i8+i32", "i32+i32", "i32+i8"])
@pytest.mark.parametrize("ngroups,lds", [(3, 0), (75, 0), (5000, 0), (200_000, 0), (75, -1),
                                         (5000, -1)])
def test_groupby(key_dtypes, ngroups, lds):
    r = rng(ngroups + 10 * len(key_dtypes))
    n = 150_001
    keys, vals = groupby_inputs(r, n, key_dtypes, ngroups)
    announce("groupby", [np.dtype(d).name for d in key_dtypes], ngroups, lds)
    t = rel.tuning(lds_slots=lds)
    got = rel.groupby_agg([dev(k) for k in keys], [dev(v) for v in vals], ALL_AGGS,
                          max_groups=min(n, ngroups ** max(1, len(key_dtypes))), t=t)
    assert_groups(got, oracle.groupby(keys, vals, ALL_AGGS), ALL_AGGS,
                  f"groupby {key_dtypes} {ngroups}")


def test_groupby_sentinel_patterns():
    announce("groupby sentinel keys")
    r = rng(5)
    n = 20_000
    v = r.integers(-50, 50, size=n).astype(np.int64)
    k64 = r.choice(np.array([I64_MIN, I64_MAX, -1, 0, 3], dtype=np.int64), size=n)
    aggs = [("sum", 0), ("count", None), ("avg", 0), ("max", 0)]
    got = rel.groupby_agg([dev(k64)], [dev(v)], aggs, max_groups=16)
    assert_groups(got, oracle.groupby([k64], [v], aggs), aggs, "int64 sentinel")
    # (INT32_MIN, 0) packs to the sentinel pattern of two int32 keys
    a = r.choice(np.array([I32_MIN, 0, 1], dtype=np.int32), size=n)
    b = r.choice(np.array([0, I32_MIN, -1], dtype=np.int32), size=n)
    got = rel.groupby_agg([dev(a), dev(b)], [dev(v)], aggs, max_groups=16)
    assert_groups(got, oracle.groupby([a, b], [v], aggs), aggs, "int32 pair sentinel")


def test_groupby_empty_inputs():
    announce("groupby empty")
    aggs = [("sum", 0), ("count", None), ("min", 0), ("max", 0), ("avg", 0)]
    e32, e64 = np.zeros(0, np.int32), np.zeros(0, np.int64)
    got = rel.groupby_agg([dev(e32)], [dev(e64)], aggs, max_groups=8)
    assert got[1][0].numel() == 0
    got = rel.groupby_agg([], [dev(e64)], aggs, max_groups=1)
    assert_groups(got, oracle.groupby([], [e64], aggs), aggs, "ungrouped empty")


def test_groupby_too_many_groups():
    announce("groupby overflow")
    k = np.arange(10_000, dtype=np.int32)
    v = np.ones(10_000, np.int64)
    with pytest.raises(rel.RelError) as e:
        rel.groupby_agg([dev(k)], [dev(v)], [("sum", 0)], max_groups=1)
    assert e.value.status == rel.REL_ECAPACITY


def test_groupby_with_row_ids():
    announce("groupby idx")
    r = rng(6)
    n = 100_000
    k = r.integers(0, 300, size=n).astype(np.int32)
    v = r.integers(0, 10**6, size=n).astype(np.int64)
    sel = r.permutation(n)[: n // 2].astype(np.uint32)
    aggs = [("sum", 0), ("count", None), ("avg", 0)]
    si = dev(sel.view(np.int32))
    got = rel.groupby_agg([dev(k)], [dev(v)], aggs, max_groups=300, key_idx=si, val_idx=si)
    assert_groups(got, oracle.groupby([k[sel]], [v[sel]], aggs), aggs, "idx")


# ------------------------------------------------- partitioned group-by

PAIR_AGGS = [("sum", 0), ("count", None), ("avg", 0), ("min", 0), ("max", 0)]


def partitioned_run(fn):
    """fn() with the kernel profiler on; asserts that the partitioning passes ran."""
    rel.profile_enable(True)
    try:
        out = fn()
        prof = rel.profile_read()
    finally:
        rel.profile_enable(False)
    assert prof["group_partition"][1] > 0, "the partitioned aggregation did not run"
    return out


@pytest.mark.parametrize("key_dtypes,ngroups,fanout,lds", [
    ([np.int32], 5000, 64, 0),
    ([np.int64], 200_000, 16384, 0),
    ([np.int64], 200_000, 4, -1),        # partitions far beyond an LDS table
    ([np.int8, np.int32], 5000, 256, 256),  # with the first scatter's LDS table
    ([np.int32, np.int32], 200_000, 1024, -1),
    ([np.int32, np.int8], 3, 16, 0),
], ids=["i32-5k-f64", "i64-200k-f16384", "i64-200k-f4-nolds", "i8+i32-5k-f256",
        "i32+i32-200k-f1024-nolds", "i32+i8-3-f16"])
def test_groupby_partitioned(key_dtypes, ngroups, fanout, lds):
    """Radix-partitioned aggregation forced by the fan-out, over keys of
    every width and three value columns (four-word records)."""
    r = rng(ngroups + 7 * fanout)
    n = 150_001
    keys, vals = groupby_inputs(r, n, key_dtypes, ngroups)
    announce("groupby partitioned", [np.dtype(d).name for d in key_dtypes], ngroups, fanout, lds)
    t = rel.tuning(lds_slots=lds, fanout=fanout)
    got = partitioned_run(lambda: rel.groupby_agg(
        [dev(k) for k in keys], [dev(v) for v in vals], ALL_AGGS,
        max_groups=min(n, ngroups ** len(key_dtypes)), t=t))
    assert_groups(got, oracle.groupby(keys, vals, ALL_AGGS), ALL_AGGS,
                  f"partitioned groupby {key_dtypes} {ngroups} fanout {fanout}")


@pytest.mark.parametrize("n,fanout,lds", [(1, 16, 0), (8192, 64, 64), (8193, 64, -1),
                                          (300_001, 4, -1), (1_000_003, 0, 0)])
def test_groupby_partitioned_skew(n, fanout, lds):
    """Zipf(1) int64 keys over 1M ranks and one value column (two-word
    records): hot keys stay in the first scatter's LDS table and the tail is
    partitioned; at fan-out 4 without that table a partition exceeds one
    aggregation piece (65536 records); fan-out 0 with 3M groups takes the
    automatic path (a group table above 64 MB)."""
    seed = 90 + n
    ranks = datagen.zipf_ranks(seed, 1, 1_000_000, 1.0, n)
    k = ((ranks * 2654435761) % (1 << 40) - (1 << 39)).astype(np.int64)
    v = datagen.uniform(seed, 2, -10**9, 10**9, n, np.int64)
    announce("groupby partitioned skew", n, fanout, lds)
    t = rel.tuning(lds_slots=lds, fanout=fanout)
    got = partitioned_run(lambda: rel.groupby_agg(
        [dev(k)], [dev(v)], PAIR_AGGS, max_groups=3_000_000 if fanout == 0 else n, t=t))
    assert_groups(got, oracle.groupby([k], [v], PAIR_AGGS), PAIR_AGGS,
                  f"partitioned skew n={n} fanout={fanout}")


def test_groupby_partitioned_sentinels_idx_overflow():
    announce("groupby partitioned sentinel/idx/overflow")
    r = rng(9)
    n = 60_000
    v = r.integers(-50, 50, size=n).astype(np.int64)
    k64 = r.integers(-5000, 5000, size=n).astype(np.int64)
    pick = r.random(n) < 0.2
    k64[pick] = r.choice(np.array([I64_MIN, I64_MAX, -1, 0], dtype=np.int64), size=int(pick.sum()))
    got = partitioned_run(lambda: rel.groupby_agg([dev(k64)], [dev(v)], PAIR_AGGS, max_groups=n,
                                                  t=rel.tuning(fanout=16)))
    assert_groups(got, oracle.groupby([k64], [v], PAIR_AGGS), PAIR_AGGS, "partitioned sentinel")
    # gathered columns
    sel = r.permutation(n)[: n // 2].astype(np.uint32)
    si = dev(sel.view(np.int32))
    got = partitioned_run(lambda: rel.groupby_agg([dev(k64)], [dev(v)], PAIR_AGGS, max_groups=n,
                                                  key_idx=si, val_idx=si,
                                                  t=rel.tuning(fanout=64)))
    assert_groups(got, oracle.groupby([k64[sel]], [v[sel]], PAIR_AGGS), PAIR_AGGS,
                  "partitioned idx")
    # more distinct keys than the table sized for max_groups holds
    k = np.arange(10_000, dtype=np.int32)
    with pytest.raises(rel.RelError) as e:
        rel.groupby_agg([dev(k)], [dev(np.ones(10_000, np.int64))], [("sum", 0)], max_groups=1,
                        t=rel.tuning(fanout=4))
    assert e.value.status == rel.REL_ECAPACITY


def test_groupby_partitioned_matches_single_pass():
    """The same call with and without partitioning, COUNT only (one-word
    records) and a pair of int32 keys: identical groups."""
    announce("groupby partitioned vs single pass")
    r = rng(12)
    n = 500_000
    a = r.integers(0, 700, size=n).astype(np.int32)
    b = r.integers(0, 700, size=n).astype(np.int32)
    aggs = [("count", None)]
    one = rel.groupby_agg([dev(a), dev(b)], [], aggs, max_groups=n, t=rel.tuning(fanout=-1))
    two = partitioned_run(lambda: rel.groupby_agg([dev(a), dev(b)], [], aggs, max_groups=n,
                                                  t=rel.tuning(fanout=512)))
    assert_groups(two, oracle.groupby([a, b], [], aggs), aggs, "partitioned count")
    assert_groups(one, oracle.groupby([a, b], [], aggs), aggs, "single-pass count")


# ---------------------------------------------------------------- pipeline

STAR_AGGS = [("sum", 3), ("count", None), ("avg", 3), ("min", 3), ("max", 3)]


def star_plan(d):
    fact = [d["fk_a"], d["fk_b"], d["date"], d["price"], d["flag"]]
    dims = [dict(fk=0, key=d["dim_a_key"], payload=None),
            dict(fk=1, key=d["dim_b_key"], payload=d["dim_b_region"])]
    return fact, [(2, "lt", 767)], dims, [("dim", 1), ("fact", 4)], STAR_AGGS


def run_both(fact, terms, dims, keys, aggs, max_groups, t=None):
    ddims = [dict(fk=x["fk"], key=dev(x["key"]),
                  payload=None if x.get("payload") is None else dev(x["payload"])) for x in dims]
    got = rel.pipeline([dev(c) for c in fact], terms, ddims, keys, aggs, max_groups, t)
    want = oracle.pipeline(fact, terms, dims, keys, aggs)
    return got, want


@pytest.mark.parametrize("n", [0, 1, 4095, 4097, 300_001])
def test_pipeline_star_schema(n):
    announce("pipeline star", n)
    d = datagen.star_schema(seed=11, n_fact=n, n_dim_a=30_000, n_dim_b=2_000)
    fact, terms, dims, keys, aggs = star_plan(d)
    got, want = run_both(fact, terms, dims, keys, aggs, max_groups=128)
    assert_groups(got, want, aggs, f"star {n}")


@pytest.mark.parametrize("lds", [0, -1])
def test_pipeline_dims_with_duplicates_and_sentinels(lds):
    announce("pipeline dup dims", lds)
    r = rng(21)
    n = 60_000
    fk0 = r.choice(np.array([I32_MIN, -1, 0, 1, 2, 3, 4, 5], dtype=np.int32), size=n)
    fk1 = r.integers(-2, 40, size=n).astype(np.int64)
    date = r.integers(0, 100, size=n).astype(np.int32)
    price = col_with_extremes(r, n, np.int64, -10**9, 10**9, 0.01)
    flag = r.integers(0, 3, size=n).astype(np.int8)
    fact = [fk0, fk1, date, price, flag]
    dims = [dict(fk=0, key=np.array([I32_MIN, 0, 0, 1, 3, 3, 3, 9], np.int32),
                 payload=np.array([7, -1, 2, 2, 5, -128, 0, 1], np.int8)),
            dict(fk=1, key=r.integers(-2, 30, size=50).astype(np.int64),
                 payload=r.integers(-5, 5, size=50).astype(np.int32))]
    keys = [("dim", 0), ("fact", 4)]
    got, want = run_both(fact, [(2, "range", 10, 70), (3, "ne", 0)], dims, keys, STAR_AGGS,
                         max_groups=256, t=rel.tuning(lds_slots=lds))
    assert_groups(got, want, STAR_AGGS, "dup dims")


def test_pipeline_shapes():
    r = rng(22)
    n = 80_000
    a = r.integers(0, 50_000, size=n).astype(np.int32)
    g = r.integers(0, 1000, size=n).astype(np.int32)
    v = r.integers(-10**6, 10**6, size=n).astype(np.int64)
    fact = [a, g, v]
    aggs = [("sum", 2), ("count", None), ("max", 2)]
    big_dim = dict(fk=0, key=r.permutation(60_000).astype(np.int32),
                   payload=r.integers(0, 70_000, size=60_000).astype(np.int32))
    dup_member = dict(fk=0, key=r.integers(0, 40_000, size=30_000).astype(np.int32), payload=None)
    uniq_member = dict(fk=1, key=r.permutation(800).astype(np.int32), payload=None)
    cases = {
        "no dims, fact key": ([], [("fact", 1)], [(2, "gt", 0)]),
        "no dims, no keys": ([], [], [(2, "gt", 0)]),
        "no predicate": ([big_dim], [("dim", 0)], []),
        "HBM dim, dim key": ([big_dim], [("dim", 0)], [(1, "lt", 500)]),
        "dim key + fact key": ([big_dim], [("dim", 0), ("fact", 1)], [(1, "lt", 500)]),
        "membership dim with duplicate keys": ([dup_member], [("fact", 1)], [(1, "lt", 900)]),
        "two membership dims": ([dup_member, uniq_member], [("fact", 1)], []),
    }
    for name, (dims, keys, terms) in cases.items():
        announce("pipeline shape", name)
        got, want = run_both(fact, terms, dims, keys, aggs, max_groups=80_000)
        assert_groups(got, want, aggs, name)


@pytest.mark.parametrize("direct", [True, False])
def test_pipeline_many_accumulators(direct):
    """Eight accumulators over four value columns of three widths through the
    fused pipeline: the first two distinct value columns are gathered with
    the keys, the other two loaded late, and the update loop walks the whole
    packed accumulator plan. With dense dim keys the direct-table kernel does
    the work, with direct tables switched off the general one (HBM map)."""
    announce("pipeline many accumulators", direct)
    r = rng(31 if direct else 32)
    n = 70_001
    key = r.permutation(5_000).astype(np.int32)
    pay = r.integers(0, 40, size=5_000).astype(np.int32)
    fk = r.integers(-100, 5_100, size=n).astype(np.int32)
    v0 = col_with_extremes(r, n, np.int64, -10**12, 10**12, 0.01)
    v1 = col_with_extremes(r, n, np.int32, -10**6, 10**6, 0.01)
    v2 = r.integers(-128, 128, size=n).astype(np.int8)
    v3 = col_with_extremes(r, n, np.int64, -10**9, 10**9, 0.01)
    flag = r.integers(0, 3, size=n).astype(np.int8)
    fact = [fk, v0, v1, v2, v3, flag]
    dims = [dict(fk=0, key=key, payload=pay)]
    # eight aggregates, eight accumulators (AVG adds the sum of its column;
    # the row count is always kept)
    aggs = [("sum", 1), ("min", 2), ("max", 3), ("sum", 4), ("max", 1), ("min", 4), ("sum", 3),
            ("avg", 2)]
    keys = [("dim", 0), ("fact", 5)]
    terms = [(5, "lt", 2)]
    t = rel.tuning(dim_lds_bytes=-1, flags=0 if direct else rel.TUNE_NO_DIRECT)
    got, want = run_both(fact, terms, dims, keys, aggs, max_groups=256, t=t)
    assert_groups(got, want, aggs, f"many accumulators direct={direct}")


def test_pipeline_int64_dim_keys():
    announce("pipeline int64 dims")
    d = datagen.skewed(n_build=20_000, n_probe=200_000, n_groups=500)
    fact = [d["probe_key"], d["probe_grp"], d["probe_val"]]
    dims = [dict(fk=0, key=d["build_key"], payload=None)]
    aggs = [("sum", 2), ("count", None)]
    got, want = run_both(fact, [], dims, [("fact", 1)], aggs, max_groups=1000)
    assert_groups(got, want, aggs, "int64 dims")


# ------------------------------------------------------------ workload sizes

def test_join_groupby_workload_full_size():
    """65,536 build rows x 1,048,576 probe rows, SUM/COUNT by a 64-value
    build attribute: as the fused plan, and as join -> group-by chained
    through row ids."""
    announce("join+groupby 64k x 1M")
    d = datagen.join_groupby()
    fact = [d["probe_key"], d["probe_val"]]
    dims = [dict(fk=0, key=d["build_key"], payload=d["build_grp"])]
    aggs = [("sum", 1), ("count", None)]
    got, want = run_both(fact, [], dims, [("dim", 0)], aggs, max_groups=64)
    assert_groups(got, want, aggs, "fused")
    # chained: pairs -> gather build attribute and probe value by row id
    ob, op = rel.hash_join(dev(d["build_key"]), dev(d["probe_key"]))
    assert_pairs((ob, op), oracle.hash_join(d["build_key"], d["probe_key"]), "join")
    chained_aggs = [("sum", 0), ("count", None)]
    got2 = rel.groupby_agg([dev(d["build_grp"])], [dev(d["probe_val"])], chained_aggs,
                           max_groups=64, key_idx=ob, val_idx=op)
    assert_groups(got2, want, chained_aggs, "chained")


def _fmix32_inverse(h):
    """Inverse of the MurmurHash3 32-bit finaliser (test-side, to craft keys
    whose hashes fall in one bucket of a compact membership set)."""
    m = 0xFFFFFFFF
    h ^= h >> 16
    h = (h * pow(0xC2B2AE35, -1, 2**32)) & m
    h ^= (h >> 13) ^ (h >> 26)
    h = (h * pow(0x85EBCA6B, -1, 2**32)) & m
    h ^= h >> 16
    return h


def test_pipeline_large_membership_dim():
    """A membership dim large enough for the 16-bit compact set (> 786k keys),
    with duplicate keys and 40 keys crafted to share one bucket, so that
    displaced entries and the out-of-band list are exercised."""
    announce("pipeline compact membership dim")
    r = rng(31)
    nd = 900_000
    keys = r.choice(2**31 - 1, size=nd, replace=False).astype(np.int64) - 2**30
    bucket = 12345
    crafted = []
    for rem in range(40):
        k = _fmix32_inverse((bucket << 14) | rem)
        crafted.append(k - 2**32 if k >= 2**31 else k)
    keys = np.concatenate([keys, np.array(crafted, np.int64), keys[:500]])  # + 500 duplicates
    dim_key = keys.astype(np.int32)
    n = 400_000
    fk = np.concatenate([r.choice(dim_key, size=n - 2000), r.integers(-2**31, 2**31 - 1, size=1000),
                         np.repeat(np.array(crafted, np.int64), 25)]).astype(np.int32)
    r.shuffle(fk)
    g = r.integers(0, 50, size=n).astype(np.int32)
    v = r.integers(-10**6, 10**6, size=n).astype(np.int64)
    fact = [fk, g, v]
    dims = [dict(fk=0, key=dim_key, payload=None)]
    aggs = [("sum", 2), ("count", None), ("min", 2)]
    got, want = run_both(fact, [], dims, [("fact", 1)], aggs, max_groups=64)
    assert_groups(got, want, aggs, "compact set")


@pytest.mark.parametrize("dim_lds", [-1, 0])
def test_pipeline_unique_compact_set_star_shape(dim_lds):
    """The star plan's shape (date predicate, a membership dim, a payload dim,
    keys from the payload and an int8 column, four aggregates over one int64
    column) with a unique 900k-key membership dim in hash tables: the plan
    runs the specialised kernel, whose compact-set probe tests a bucket's
    eight entries at once. 40 crafted keys share one home bucket, so probes
    walk the displaced entries and the overflow set; fact keys mix members,
    non-members and the crafted keys. With the default dim LDS budget the
    1000-key payload dim is copied into LDS and the general kernel runs."""
    announce("pipeline unique compact set, star shape", dim_lds)
    r = rng(32)
    nd = 900_000
    crafted = []
    for rem in range(40):
        k = _fmix32_inverse((777 << 14) | rem)
        crafted.append(k - 2**32 if k >= 2**31 else k)
    keys = r.choice(2**31 - 1, size=nd + 200, replace=False).astype(np.int64) - 2**30
    keys = np.setdiff1d(keys, np.array(crafted, np.int64))[:nd]
    r.shuffle(keys)
    dim_a = np.concatenate([keys, np.array(crafted, np.int64)]).astype(np.int32)
    nb = 1000
    dim_b = r.choice(2**31 - 1, size=nb, replace=False).astype(np.int32)
    region = r.integers(0, 5, size=nb).astype(np.int32)
    n = 300_001
    fk_a = np.concatenate([r.choice(dim_a, size=n - 3000), r.integers(-2**31, 2**31 - 1, size=2000),
                           np.repeat(np.array(crafted, np.int64), 25)]).astype(np.int32)
    r.shuffle(fk_a)
    fk_b = r.choice(dim_b, size=n)
    fk_b[r.random(n) < 0.05] = -7  # not a dim-B key
    date = r.integers(0, 2557, size=n).astype(np.int32)
    price = r.integers(-10**9, 10**9, size=n).astype(np.int64)
    flag = r.integers(0, 3, size=n).astype(np.int8)
    fact = [fk_a, fk_b, date, price, flag]
    dims = [dict(fk=0, key=dim_a, payload=None), dict(fk=1, key=dim_b, payload=region)]
    aggs = [("sum", 3), ("count", None), ("avg", 3), ("min", 3), ("max", 3)]
    t = rel.tuning(flags=rel.TUNE_NO_DIRECT, dim_lds_bytes=dim_lds)
    got, want = run_both(fact, [(2, "lt", 2000)], dims, [("dim", 1), ("fact", 4)], aggs,
                         max_groups=64, t=t)
    assert_groups(got, want, aggs, "unique compact set")


def _direct_case(r, name, n_dim=20_000, n_fact=150_000):
    """A dim with int32 keys laid out to reach one path of the direct
    tables: the full key range, a partial range (presence bitmap), payload
    spans of 1, 2 and 4 bytes, keys at the int32 extremes, duplicates (back
    to the hash table) and a range too wide for a direct table."""
    base = {"full": 1_000, "partial": -7_000, "wide_payload": 0, "extreme_low": -(2**31),
            "extreme_high": 2**31 - n_dim, "dups": 50, "too_wide": 0}[name]
    if name == "partial":
        key = (r.choice(2 * n_dim, size=n_dim, replace=False) + base).astype(np.int64)
    elif name == "too_wide":
        key = r.choice(50 * n_dim, size=n_dim, replace=False).astype(np.int64)
    else:
        key = r.permutation(n_dim).astype(np.int64) + base
    if name == "dups":
        key[:300] = key[300:600]
    payload = {"wide_payload": r.integers(-2**31, 2**31 - 1, size=n_dim),
               "partial": r.integers(-500, 40_000, size=n_dim)}.get(
        name, r.integers(-3, 20, size=n_dim)).astype(np.int32)
    lo, hi = int(key.min()) - 50, int(key.max()) + 50
    fk = np.where(r.random(n_fact) < 0.8, r.choice(key, size=n_fact),
                  r.integers(max(lo, -(2**31)), min(hi, 2**31 - 1), size=n_fact))
    return key.astype(np.int32), payload, fk.astype(np.int32)


@pytest.mark.parametrize("name", ["full", "partial", "wide_payload", "extreme_low",
                                  "extreme_high", "dups", "too_wide"])
def test_pipeline_direct_dims(name):
    announce("pipeline direct dims", name)
    r = rng(sum(map(ord, name)))
    key0, pay0, fk0 = _direct_case(r, name)
    # a second, membership-only dim over a dense range as well
    key1 = r.permutation(3_000).astype(np.int32) + 17
    fk1 = r.integers(0, 3_100, size=len(fk0)).astype(np.int32)
    g = r.integers(0, 5, size=len(fk0)).astype(np.int32)
    v = col_with_extremes(r, len(fk0), np.int64, -10**9, 10**9, 0.01)
    fact = [fk0, fk1, g, v]
    dims = [dict(fk=0, key=key0, payload=pay0), dict(fk=1, key=key1, payload=None)]
    aggs = [("sum", 3), ("count", None), ("min", 3), ("max", 3), ("avg", 3)]
    keys = [("dim", 0), ("fact", 2)]
    want = oracle.pipeline(fact, [(2, "ne", 3)], dims, keys, aggs)
    for t in (None, rel.tuning(flags=rel.TUNE_NO_DIRECT), rel.tuning(dim_lds_bytes=-1)):
        got, _ = run_both(fact, [(2, "ne", 3)], dims, keys, aggs, max_groups=200_000, t=t)
        assert_groups(got, want, aggs, f"direct {name} tuning {t and t.flags}")
