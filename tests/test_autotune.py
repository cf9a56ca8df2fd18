"""Autotuner host logic: size buckets, the JSON cache, candidate records."""

import json

import pytest

from paper_2508_04701_amd import autotune, rel


def test_buckets_group_sizes_by_magnitude():
    assert autotune.bucket(1, 0, 1) == "f0-d0-g0"
    assert autotune.bucket(1000, 1000, 8) == autotune.bucket(900, 600, 5)
    assert autotune.bucket(4096, 100, 64) != autotune.bucket(4097 * 4, 100, 64)
    b = autotune.bucket(600_000_000, 1_500_000, 75)
    assert b == "f30-d20-g6"


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    c = autotune.Cache(path)
    key = autotune.cache_key("join_groupby", autotune.bucket(10**6, 10**4, 500), gpu="gfx950")
    c.put(key, {"tuning": {"replicas": 32}, "ms": 1.5, "candidates": {"{}": 2.0}})
    c.save()
    d = autotune.Cache(path)
    assert d.get(key) == {"replicas": 32}
    assert d.get("gfx950/join_groupby/none") is None
    assert json.load(open(path))[key]["ms"] == 1.5


def test_every_candidate_is_a_valid_tuning():
    L = rel.lib()
    for cand in autotune.CANDIDATES:
        t = autotune.to_tuning(cand)
        if t is None:
            continue
        # a valid record: the library accepts it for a plan's workspace size
        n = L.rel_hash_join_ws(2, 1000, rel.ctypes.byref(t))
        assert n > 0, cand
    kt = (rel.ctypes.c_int32 * 1)(3)
    aggs = (rel.Agg * 1)(rel.Agg(0, 0))
    for cand in autotune.GROUPBY_CANDIDATES:
        t = autotune.to_tuning(cand)
        if t is None:
            continue
        assert L.rel_groupby_ws(1, kt, 1, aggs, 1_000_000, 200_000, rel.ctypes.byref(t)) > 0, cand
    with pytest.raises(ValueError):
        autotune.to_tuning({"warp_size": 32})
