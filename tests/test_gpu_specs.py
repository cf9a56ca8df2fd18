"""The specialised fused kernels (compile-time row specs) against the oracle:
every built spec (a dim-1 payload and an int8 fact column as keys; one dim
payload as key) over hash-table dims held in HBM, with each predicate form
the host folds into a range (lt, le, gt, ge, eq, range, none) at the int32
boundaries and beyond them, sentinel foreign and dim keys, ragged tails, and
the cases that must fall back to the generic kernel (a ne term, duplicate dim
keys, a misaligned column, direct tables) - all bit-exact."""

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import announce, assert_groups, dev
from paper_2508_04701_amd import datagen, rel

pytestmark = pytest.mark.gpu

I32_MIN, I32_MAX = -(2**31), 2**31 - 1
HASH = rel.tuning(flags=rel.TUNE_NO_DIRECT, dim_lds_bytes=-1)
STAR_AGGS = [("sum", 3), ("count", None), ("avg", 3), ("min", 3), ("max", 3)]


def run(fact, terms, dims, keys, aggs, max_groups, t=HASH, fact_dev=None):
    ddims = [dict(fk=x["fk"], key=dev(x["key"]),
                  payload=None if x.get("payload") is None else dev(x["payload"])) for x in dims]
    fd = fact_dev if fact_dev is not None else [dev(c) for c in fact]
    got = rel.pipeline(fd, terms, ddims, keys, aggs, max_groups, t)
    want = oracle.pipeline(fact, terms, dims, keys, aggs)
    return got, want


def star(n, seed, n_dim_a=30_000, n_dim_b=2_000):
    d = datagen.star_schema(seed=seed, n_fact=n, n_dim_a=n_dim_a, n_dim_b=n_dim_b)
    fact = [d["fk_a"], d["fk_b"], d["date"], d["price"], d["flag"]]
    dims = [dict(fk=0, key=d["dim_a_key"], payload=None),
            dict(fk=1, key=d["dim_b_key"], payload=d["dim_b_region"])]
    return fact, dims


@pytest.mark.parametrize("n", [1, 3, 2048, 4095, 4097, 2048 * 37 + 3, 400_000])
def test_spec_star_sizes(n):
    announce("spec star", n)
    fact, dims = star(n, 41)
    got, want = run(fact, [(2, "lt", 767)], dims, [("dim", 1), ("fact", 4)], STAR_AGGS, 128)
    assert_groups(got, want, STAR_AGGS, f"spec star {n}")


TERMS = {
    "lt": (2, "lt", 767), "le": (2, "le", 766), "gt": (2, "gt", 1500), "ge": (2, "ge", 1500),
    "eq": (2, "eq", 42), "range": (2, "range", 300, 900), "lt_min": (2, "lt", I32_MIN),
    "le_min": (2, "le", I32_MIN), "lt_beyond": (2, "lt", 2**40), "ge_beyond": (2, "ge", -(2**40)),
    "gt_max": (2, "gt", I32_MAX), "ge_max": (2, "ge", I32_MAX), "le_max": (2, "le", I32_MAX),
    "eq_beyond": (2, "eq", 2**33), "eq_min": (2, "eq", I32_MIN), "range_wide": (2, "range", -(2**40), 2**40),
    "range_empty": (2, "range", 500, 400), "ne": (2, "ne", 7), "none": None,
}


@pytest.mark.parametrize("name", sorted(TERMS))
def test_spec_predicate_forms(name):
    announce("spec predicate", name)
    r = np.random.default_rng(sum(map(ord, name)))
    fact, dims = star(50_003, 43)
    date = fact[2].copy()
    # extremes of the int32 domain in the predicate column
    pick = r.choice(len(date), size=300, replace=False)
    date[pick[:100]] = I32_MIN
    date[pick[100:200]] = I32_MAX
    date[pick[200:]] = 42
    fact[2] = date
    term = TERMS[name]
    terms = [] if term is None else [term]
    got, want = run(fact, terms, dims, [("dim", 1), ("fact", 4)], STAR_AGGS, 128)
    assert_groups(got, want, STAR_AGGS, f"predicate {name}")


def test_spec_sentinel_keys_and_misses():
    """Foreign keys equal to the hash tables' empty sentinel (INT32_MIN) and
    keys that miss; the dims hold the sentinel as a real key."""
    announce("spec sentinel keys")
    r = np.random.default_rng(44)
    fact, dims = star(120_000, 45, n_dim_a=20_000, n_dim_b=3_000)
    fk_a, fk_b = fact[0].copy(), fact[1].copy()
    fk_a[r.choice(len(fk_a), 500, replace=False)] = I32_MIN
    fk_b[r.choice(len(fk_b), 700, replace=False)] = I32_MIN
    fk_a[r.choice(len(fk_a), 900, replace=False)] = 10**9  # misses
    fk_b[r.choice(len(fk_b), 900, replace=False)] = -5      # misses
    fact[0], fact[1] = fk_a, fk_b
    ka, kb = dims[0]["key"].copy(), dims[1]["key"].copy()
    ka[7] = I32_MIN
    kb[11] = I32_MIN
    dims[0]["key"], dims[1]["key"] = ka, kb
    got, want = run(fact, [(2, "lt", 1200)], dims, [("dim", 1), ("fact", 4)], STAR_AGGS, 128)
    assert_groups(got, want, STAR_AGGS, "sentinels")


def test_spec_join_groupby_shapes():
    """One dim-payload key (dim 0, and dim 1 of a two-dim plan), SUM/COUNT
    and MIN/MAX over an int64 column."""
    d = datagen.join_groupby(n_build=20_000, n_probe=300_001, n_groups=64, probe_domain=22_000)
    fact = [d["probe_key"], d["probe_val"]]
    dims = [dict(fk=0, key=d["build_key"], payload=d["build_grp"])]
    for aggs in ([("sum", 1), ("count", None)], [("min", 1), ("max", 1), ("avg", 1)]):
        announce("spec join+groupby", aggs)
        got, want = run(fact, [], dims, [("dim", 0)], aggs, 64)
        assert_groups(got, want, aggs, f"dim0 key {aggs}")
    fact2, dims2 = star(200_000, 46)
    announce("spec dim1 key")
    got, want = run(fact2, [(2, "ge", 2000)], dims2, [("dim", 1)], STAR_AGGS, 64)
    assert_groups(got, want, STAR_AGGS, "dim1 key")


def test_spec_falls_back_to_generic():
    """Plans of a specialised shape that the generic kernel must take:
    duplicate dim keys (decided on the device), a misaligned fact column,
    and the same plans with direct tables allowed."""
    fact, dims = star(150_000, 47, n_dim_a=20_000, n_dim_b=3_000)
    keys = [("dim", 1), ("fact", 4)]
    terms = [(2, "lt", 900)]
    dup = [dict(dims[0]), dict(dims[1])]
    kb = dup[1]["key"].copy()
    kb[:40] = kb[40:80]
    dup[1]["key"] = kb
    for name, dm, t in (("dup dim keys", dup, HASH), ("dup dim keys, direct allowed", dup, None),
                        ("direct tables", dims, None)):
        announce("spec fallback", name)
        got, want = run(fact, terms, dm, keys, STAR_AGGS, 128, t=t)
        assert_groups(got, want, STAR_AGGS, name)
    announce("spec fallback misaligned")
    # fk_a stored one element into a larger buffer: its data pointer is not
    # 16-byte aligned, so the specialised loads do not apply
    buf = torch.empty(len(fact[0]) + 1, dtype=torch.int32, device="cuda")
    buf[1:] = dev(fact[0])
    fd = [buf[1:]] + [dev(c) for c in fact[1:]]
    got, want = run(fact, terms, dims, keys, STAR_AGGS, 128, fact_dev=fd)
    assert_groups(got, want, STAR_AGGS, "misaligned")
