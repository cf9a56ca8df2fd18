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


class _HostPlan:
    """Just a rel_pipeline_desc over host-side fake pointers (lookups only
    read sizes)."""

    def __init__(self, n_fact, n_dim, max_groups):
        self.fact = (rel.Column * 1)(rel.Column(0x1000, None, n_fact, 2, 0))
        self.dims = (rel.Dim * 1)(rel.Dim(0, 0, rel.Column(0x2000, None, n_dim, 2, 0), rel.Column()))
        self.aggs = (rel.Agg * 1)(rel.Agg(1, 0))
        self.desc = rel.PipelineDesc(rel.ctypes.cast(self.fact, rel.ctypes.POINTER(rel.Column)), 1,
                                     None, 0, rel.ctypes.cast(self.dims, rel.ctypes.POINTER(rel.Dim)),
                                     1 if n_dim else 0, None, 0,
                                     rel.ctypes.cast(self.aggs, rel.ctypes.POINTER(rel.Agg)), 1,
                                     max_groups, None)


def test_native_lookup_reads_python_written_records(tmp_path):
    """rel_autotune_lookup finds the record of a plan's bucket (same bucket
    rule as autotune.bucket) in a cache written by the Python side; on a
    machine without a GPU the architecture is "none"."""
    path = str(tmp_path / "tune.json")
    c = autotune.Cache(path)
    b = autotune.bucket(5_000_000, 300_000, 5_000)
    c.put(f"none/pipeline_batch/{b}", {"tuning": {"replicas": 32, "load_factor": 0.3,
                                                 "chunk_tiles": 4, "grid": 256},
                                      "ms": 1.0, "candidates": {}})
    c.put("none/groupby/f0-d0-g0", {"tuning": {"fanout": 8192}, "ms": 2.0, "candidates": {}})
    c.save()
    t = autotune.lookup(path, _HostPlan(5_000_000, 300_000, 5_000))
    assert t is not None
    assert (t.replicas, t.chunk_tiles, t.grid) == (32, 4, 256)
    assert abs(t.load_factor - 0.3) < 1e-6 and t.lds_slots == 0
    # another bucket (fact rows 16x larger): no record
    assert autotune.lookup(path, _HostPlan(80_000_000, 300_000, 5_000)) is None
    # a missing cache file is an empty cache
    assert autotune.lookup(str(tmp_path / "none.json"), _HostPlan(10, 10, 10)) is None


def test_native_lookup_rejects_bad_records(tmp_path):
    path = str(tmp_path / "bad.json")
    b = autotune.bucket(1000, 100, 10)
    with open(path, "w") as f:
        json.dump({f"none/pipeline_batch/{b}": {"tuning": {"warp": 32}}}, f)
    with pytest.raises(rel.RelError):
        autotune.lookup(path, _HostPlan(1000, 100, 10))
    with open(path, "w") as f:
        f.write("{not json")
    with pytest.raises(rel.RelError):
        autotune.lookup(path, _HostPlan(1000, 100, 10))


def test_native_autotune_validates_before_any_device_call(tmp_path):
    L = rel.lib()
    assert L.rel_autotune(None, 0, str(tmp_path / "x.json").encode()) == rel.REL_EINVAL
    p = _HostPlan(1000, 100, 10)
    descs = (rel.PipelineDesc * 1)(p.desc)
    assert L.rel_autotune(descs, 1, None) == rel.REL_EINVAL
    bad = _HostPlan(1000, 100, -5)
    descs = (rel.PipelineDesc * 1)(bad.desc)
    assert L.rel_autotune(descs, 1, str(tmp_path / "x.json").encode()) == rel.REL_EINVAL
