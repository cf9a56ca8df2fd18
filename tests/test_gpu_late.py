"""Late materialisation (rel_gather) and order-by / top-N (rel_topn) against
the oracle: gathers of every column width at filter- and join-shaped row
ids; top-N over group-by outputs ordered by int64 and binary64 columns,
ascending and descending, with heavy ties (broken by the key tuple, then the
position), limits from 0 to 1024, sizes across the chunk and merge-round
boundaries, and the chain group-by -> top-N -> gather."""

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import announce, dev, rowids
from paper_2508_04701_amd import rel

pytestmark = pytest.mark.gpu

I64_MIN, I64_MAX = -(2**63), 2**63 - 1


@pytest.mark.parametrize("n", [0, 1, 3, 4, 5, 1023, 100_003])
def test_gather_all_widths(n):
    announce("gather", n)
    r = np.random.default_rng(n + 1)
    m = 50_000
    cols = [r.integers(-128, 128, size=m).astype(np.int8),
            r.integers(-2**31, 2**31 - 1, size=m).astype(np.int32),
            r.integers(I64_MIN, I64_MAX, size=m, dtype=np.int64)]
    ids = r.integers(0, m, size=n).astype(np.uint32)
    got = rel.gather([dev(c) for c in cols], dev(ids.view(np.int32)))
    for c, g in zip(cols, got):
        assert np.array_equal(g.cpu().numpy().astype(np.int64), oracle.gather(c, ids))


def test_gather_after_filter_unaligned_ids():
    announce("gather after filter")
    r = np.random.default_rng(3)
    v = r.integers(0, 10**9, size=300_001).astype(np.int64)
    date = r.integers(0, 2557, size=300_001).astype(np.int32)
    ids = rel.filter([dev(date)], [(0, "lt", 767)])
    want_ids = oracle.filter([date], [(0, "lt", 767)])
    assert np.array_equal(rowids(ids), want_ids)
    # a view one element in: the ids are not 16-byte aligned
    got = rel.gather([dev(v)], ids[1:])[0].cpu().numpy()
    assert np.array_equal(got, oracle.gather(v, want_ids[1:]))


def _check_topn(order, keys, limit, desc, what):
    d_order = dev(order)
    got = rowids(rel.topn(d_order, [dev(k) for k in keys], limit, desc))
    want = oracle.topn(order, [k.astype(np.int64) for k in keys], limit, desc)
    assert np.array_equal(got, want), f"{what}: {got[:8]} vs {want[:8]}"


@pytest.mark.parametrize("n", [0, 1, 7, 1024, 1025, 513 * 1024 + 17, 3_000_001])
@pytest.mark.parametrize("limit", [0, 1, 10, 1000, 1024])
def test_topn_int64_with_ties(n, limit):
    announce("top-N int64", n, limit)
    r = np.random.default_rng(n * 31 + limit)
    order = r.integers(-50, 50, size=n).astype(np.int64)  # heavy ties
    order[r.random(n) < 0.001] = I64_MAX
    order[r.random(n) < 0.001] = I64_MIN
    k0 = r.integers(-3, 3, size=n).astype(np.int32)
    k1 = r.permutation(n).astype(np.int64)
    for desc in (True, False):
        _check_topn(order, [k0, k1], limit, desc, f"n={n} limit={limit} desc={desc}")


@pytest.mark.parametrize("nkeys", [0, 1, 2])
def test_topn_double_order(nkeys):
    announce("top-N double", nkeys)
    r = np.random.default_rng(7 + nkeys)
    n = 200_000
    order = np.round(r.normal(size=n), 2)  # ties, negatives, -0.0 and 0.0
    order[:50] = -0.0
    order[50:100] = 0.0
    keys = [r.integers(-10, 10, size=n).astype(np.int8), r.permutation(n).astype(np.int32)][:nkeys]
    for desc in (True, False):
        _check_topn(order, keys, 300, desc, f"double nkeys={nkeys} desc={desc}")


def test_groupby_topn_gather_chain():
    """ORDER BY SUM DESC LIMIT 100 over a group-by: the positions come from
    rel_topn and the rows from rel_gather; compared with the oracle's
    group-by sorted the same way."""
    announce("group-by -> top-N -> gather")
    r = np.random.default_rng(9)
    n = 2_000_000
    key = r.integers(0, 300_000, size=n).astype(np.int64)
    val = r.integers(0, 1000, size=n).astype(np.int64)
    aggs = [("sum", 0), ("count", None)]
    gk, ga = rel.groupby_agg([dev(key)], [dev(val)], aggs, max_groups=300_000)
    pos = rel.topn(ga[0], gk, 100, desc=True)
    top_keys, top_sum, top_cnt = rel.gather([gk[0], ga[0], ga[1]], pos)
    wk, (ws, wc) = oracle.groupby([key], [val], aggs)
    want = oracle.topn(ws, wk, 100, desc=True)
    assert np.array_equal(top_keys.cpu().numpy(), wk[0][want])
    assert np.array_equal(top_sum.cpu().numpy(), ws[want])
    assert np.array_equal(top_cnt.cpu().numpy(), wc[want])
