"""The synchronous forms (rel_*_sync) through the C-ABI: they return the
exact result size on the host, REL_ECAPACITY when it exceeds the output
capacity (with the first out_cap items written, as the asynchronous call
writes them) or when the groups exceed max_groups, and otherwise the same
results as the asynchronous calls and the oracle."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import announce, assert_groups, assert_pairs, dev, rowids
from paper_2508_04701_amd import rel

pytestmark = pytest.mark.gpu


def _s():
    return rel._stream()


def test_filter_sync_capacity():
    announce("filter_sync")
    x = np.arange(10_000, dtype=np.int32)
    t = dev(x)
    cols = rel._arr(rel.Column, [rel.column(t)])
    preds = rel._preds([(0, "lt", 6000)])
    ws = rel.workspace(rel.filter_ws(len(x)))
    d = torch.zeros(1, dtype=torch.int64, device="cuda")
    cnt = ctypes.c_int64(-5)
    out = torch.full((100,), -1, dtype=torch.int32, device="cuda")
    st = rel.lib().rel_filter_sync(cols, 1, preds, 1, rel._addr(out), 100, rel._addr(d),
                                   rel._addr(ws), ws.numel(), _s(), ctypes.byref(cnt))
    assert st == rel.REL_ECAPACITY and cnt.value == 6000
    assert np.array_equal(rowids(out), np.arange(100, dtype=np.uint32))
    assert np.array_equal(rowids(rel.filter([t], [(0, "lt", 6000)])), np.arange(6000, dtype=np.uint32))


def test_hash_join_sync_capacity_and_retry():
    announce("hash_join_sync")
    r = np.random.default_rng(3)
    b = r.integers(0, 50, size=200).astype(np.int32)  # duplicates: many pairs
    p = r.integers(0, 60, size=3000).astype(np.int32)
    want = oracle.hash_join(b, p)
    got = rel.hash_join(dev(b), dev(p), out_cap=7)  # first call is short, the binding retries
    assert_pairs(got, want, "join sync")
    ws = rel.workspace(rel.hash_join_ws(torch.int32, len(b)))
    ob = torch.empty(7, dtype=torch.int32, device="cuda")
    op = torch.empty(7, dtype=torch.int32, device="cuda")
    d = torch.zeros(1, dtype=torch.int64, device="cuda")
    db, dp = dev(b), dev(p)  # kept alive while the columns point into them
    cb, cp = rel.column(db), rel.column(dp)
    total = ctypes.c_int64()
    st = rel.lib().rel_hash_join_sync(ctypes.byref(cb), ctypes.byref(cp), rel._addr(ob),
                                      rel._addr(op), 7, rel._addr(d), None, rel._addr(ws),
                                      ws.numel(), _s(), ctypes.byref(total))
    assert st == rel.REL_ECAPACITY and total.value == len(want[0])


def test_groupby_sync_groups_beyond_max_groups():
    announce("groupby_sync")
    k = np.arange(5000, dtype=np.int32) % 700
    v = np.arange(5000, dtype=np.int64)
    aggs = [("sum", 0), ("count", None)]
    assert_groups(rel.groupby_agg([dev(k)], [dev(v)], aggs, max_groups=700),
                  oracle.groupby([k], [v], aggs), aggs, "groupby sync")
    with pytest.raises(rel.RelError) as e:
        rel.groupby_agg([dev(k)], [dev(v)], aggs, max_groups=100)
    assert e.value.status == rel.REL_ECAPACITY


def test_pipeline_sync_capacity():
    announce("pipeline_sync")
    r = np.random.default_rng(4)
    key = r.permutation(3000).astype(np.int32)
    pay = r.integers(0, 300, size=3000).astype(np.int32)
    fk = r.integers(0, 3000, size=50_000).astype(np.int32)
    v = r.integers(0, 10**6, size=50_000).astype(np.int64)
    dims = [dict(fk=0, key=dev(key), payload=dev(pay))]
    aggs = [("sum", 1), ("count", None)]
    plan = rel.PreparedPipeline([dev(fk), dev(v)], [], dims, [("dim", 0)], aggs, max_groups=300)
    got = plan.run()
    want = oracle.pipeline([fk, v], [], [dict(fk=0, key=key, payload=pay)], [("dim", 0)], aggs)
    assert_groups(got, want, aggs, "pipeline sync")
    small = rel.PreparedPipeline([dev(fk), dev(v)], [], dims, [("dim", 0)], aggs, max_groups=300,
                                 out_cap=10)
    with pytest.raises(rel.RelError) as e:
        small.run()
    assert e.value.status == rel.REL_ECAPACITY
