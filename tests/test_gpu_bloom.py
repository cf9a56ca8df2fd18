"""Predicate transfer: the Bloom filter built over one side's join keys and
applied to the other side (rel_bloom_build, rel_bloom_filter), and the hash
join that consults it before its table walk (REL_TUNE_BLOOM). The filter's
output is not unique (its false positives depend on the hash), so it is
checked for what is: ascending row ids, every row of the oracle's semi-join
present (no false negatives), and a false-positive share within bound. The
join with the filter must equal the oracle's join exactly, and the join of
the filtered rows reproduces the semi-join exactly."""

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import announce, assert_pairs, dev, rowids
from paper_2508_04701_amd import rel

pytestmark = pytest.mark.gpu

I32_MIN, I32_MAX = -(2**31), 2**31 - 1
I64_MIN, I64_MAX = -(2**63), 2**63 - 1


def keys_with_extremes(r, n, dtype, domain):
    k = r.integers(-domain, domain, size=n)
    ext = [I32_MIN, I32_MAX, -1, 0] if dtype == np.int32 else [I64_MIN, I64_MAX, -1, 0, I32_MIN]
    pick = r.random(n) < 0.01
    k[pick] = r.choice(ext, size=int(pick.sum()))
    return k.astype(dtype)


def check_filter(build, probe, got, bits_per_key=16):
    semi = oracle.semi_join(build, probe)
    got = np.asarray(got)
    assert np.all(np.diff(got.astype(np.int64)) > 0), "ascending row ids"
    assert np.isin(semi, got).all(), "no false negatives"
    extra = len(got) - len(semi)
    misses = len(probe) - len(semi)
    if misses > 2000:
        # about 0.1% at 16 bits per key; 0.5% leaves room for unlucky blocks
        assert extra <= 0.005 * misses + 5, f"{extra} false positives of {misses}"


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("nb,npr", [(0, 1000), (1, 1), (1000, 8191), (1000, 8193), (50_000, 600_001),
                                    (100_000, 2_100_001)])
def test_bloom_filter_semi_join_reduction(dtype, nb, npr):
    announce("bloom filter", dtype.__name__, nb, npr)
    r = np.random.default_rng(nb * 7 + npr)
    build = keys_with_extremes(r, nb, dtype, 10 * max(nb, 1))
    probe = keys_with_extremes(r, npr, dtype, 10 * max(nb, 1))
    probe[: npr // 5] = r.choice(build, size=npr // 5) if nb else probe[: npr // 5]
    f = rel.bloom_build(dev(build))
    got = rowids(rel.bloom_filter(dev(probe), f))
    check_filter(build, probe, got)


def test_bloom_filter_with_row_ids_and_mixed_widths():
    """Probe keys gathered through a selection vector; int32 build keys
    against int64 probe keys of the same values (keys compare as int64)."""
    announce("bloom filter idx / widths")
    r = np.random.default_rng(5)
    build = r.integers(-50_000, 50_000, size=20_000).astype(np.int32)
    probe = r.integers(-200_000, 200_000, size=300_000).astype(np.int64)
    sel = np.sort(r.choice(len(probe), size=100_000, replace=False)).astype(np.uint32)
    f = rel.bloom_build(dev(build))
    got = rowids(rel.bloom_filter(dev(probe), f, idx=dev(sel.view(np.int32))))
    want = sel[oracle.semi_join(build.astype(np.int64), probe[sel])]
    assert np.isin(want, got).all() and np.isin(got, sel).all()
    assert np.all(np.diff(got.astype(np.int64)) > 0)


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("fanout", [0, -1, 16])
def test_hash_join_with_bloom_filter(dtype, fanout):
    announce("join + bloom", dtype.__name__, fanout)
    r = np.random.default_rng(11 + fanout)
    nb = 200_000
    build = keys_with_extremes(r, nb, dtype, 3 * nb)
    build[:500] = build[500:1000]  # duplicates: every pair still reported
    probe = keys_with_extremes(r, 1_000_003, dtype, 30 * nb)
    probe[::10] = r.choice(build, size=len(probe[::10]))
    t = rel.tuning(flags=rel.TUNE_BLOOM, fanout=fanout)
    got = rel.hash_join(dev(build), dev(probe), t=t)
    assert_pairs(got, oracle.hash_join(build, probe), f"join with bloom {dtype.__name__}")


def test_semi_join_through_filter_and_join():
    """Exact semi-join: filter the probe side by the Bloom filter, join the
    surviving rows, keep the distinct probe rows of the pairs."""
    announce("exact semi-join")
    r = np.random.default_rng(12)
    build = r.integers(0, 10**9, size=100_000).astype(np.int64)
    probe = r.integers(0, 10**9, size=2_000_000).astype(np.int64)
    probe[::20] = r.choice(build, size=len(probe[::20]))
    db, dp = dev(build), dev(probe)
    cand = rel.bloom_filter(dp, rel.bloom_build(db))
    ob, op = rel.hash_join(db, dp, probe_idx=cand)
    semi = np.unique(rowids(op))
    assert np.array_equal(semi, oracle.semi_join(build, probe))
