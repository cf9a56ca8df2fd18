"""The C-ABI library on the CPU: it loads, exports every function that
include/rel.h declares, and rejects malformed requests on the host before any
HIP call (no GPU needed)."""

import ctypes
import os
import re

import pytest

from paper_2508_04701_amd import rel

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "rel.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(rel_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("rel_filter", "rel_hash_join", "rel_groupby_agg", "rel_pipeline"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(rel.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} not exported"
    # the binding knows every declared entry point
    assert sorted(rel.SIGNATURES) == declared_functions()


def test_version_and_status_text():
    L = rel.lib()
    assert L.rel_version() == 1
    assert L.rel_status_str(rel.REL_OK) == b"ok"
    assert L.rel_status_str(rel.REL_ENOMEM) == b"workspace too small"


def col(n, dtype=2, data=0x1000, idx=None):
    return rel.Column(data, idx, n, dtype, 0)


def call_filter(cols, preds, out_cap=10, d_count=0x2000, ws=0x10000, ws_bytes=1 << 20):
    ca = (rel.Column * max(1, len(cols)))(*cols)
    pa = (rel.Pred * max(1, len(preds)))(*preds)
    return rel.lib().rel_filter(ca, len(cols), pa, len(preds), ctypes.c_void_p(0x3000), out_cap,
                                ctypes.c_void_p(d_count), ctypes.c_void_p(ws), ws_bytes, None)


def test_filter_validation():
    L = rel.lib()
    ok_pred = rel.Pred(0, 0, 5, 0)
    assert call_filter([col(10, dtype=7)], [ok_pred]) == rel.REL_EINVAL
    assert b"invalid type" in L.rel_last_error()
    assert call_filter([col(10), col(11)], [ok_pred]) == rel.REL_EINVAL
    assert call_filter([col(10)], [rel.Pred(1, 0, 5, 0)]) == rel.REL_EINVAL
    assert call_filter([col(10)], [rel.Pred(0, 9, 5, 0)]) == rel.REL_EINVAL
    assert call_filter([col(10)], []) == rel.REL_EINVAL
    assert call_filter([col(10)], [ok_pred], d_count=0) == rel.REL_EINVAL
    assert call_filter([col(10, data=0)], [ok_pred]) == rel.REL_EINVAL
    assert call_filter([col(2**32)], [ok_pred]) == rel.REL_EUNSUPPORTED
    assert call_filter([col(10), col(10, idx=0x5000)], [ok_pred, ok_pred]) == rel.REL_EINVAL
    need = L.rel_filter_ws(10_000)
    assert call_filter([col(10_000)], [ok_pred], ws_bytes=need - 1) == rel.REL_ENOMEM
    assert call_filter([col(10_000)], [ok_pred], ws=0x10010, ws_bytes=need) == rel.REL_EINVAL


def test_workspace_sizes():
    L = rel.lib()
    assert L.rel_filter_ws(0) >= 256 + 8
    assert L.rel_filter_ws(600_000_000) >= 8 * (600_000_000 // 16384)  # a state word per tile
    small = L.rel_hash_join_ws(2, 10_000, None)
    big = L.rel_hash_join_ws(2, 1_000_000, None)
    assert 0 < small < big
    assert L.rel_hash_join_ws(3, 10_000, None) > small   # 16-byte slots for int64 keys
    assert L.rel_hash_join_ws(1, 10, None) == 0           # int8 keys are not joinable
    t = rel.tuning(load_factor=0.9, fanout=-1)
    off = rel.tuning(fanout=-1)
    assert L.rel_hash_join_ws(2, 600_000, ctypes.byref(t)) < L.rel_hash_join_ws(2, 600_000, ctypes.byref(off))
    # large build sides: the partitioned build adds two buffers of 16-byte records
    big = 100_000_000
    assert L.rel_hash_join_ws(3, big, None) >= L.rel_hash_join_ws(3, big, ctypes.byref(off)) + 32 * big
    assert L.rel_hash_join_ws(3, 1000, rel.ctypes.byref(rel.tuning(fanout=64))) == \
        L.rel_hash_join_ws(3, 1000, ctypes.byref(off))   # too small for four LDS ranges
    aggs = (rel.Agg * 2)(rel.Agg(0, 0), rel.Agg(1, 0))
    kt = (ctypes.c_int32 * 2)(2, 1)
    assert L.rel_groupby_ws(2, kt, 2, aggs, 1000, 100, None) > 0
    kt64 = (ctypes.c_int32 * 2)(3, 2)
    assert L.rel_groupby_ws(2, kt64, 2, aggs, 1000, 100, None) == 0   # 96-bit key tuple
    # many groups: the radix-partitioned path adds two buffers of n records
    # (key + one value column = 16 bytes each), unless partitioning is off
    k1 = (ctypes.c_int32 * 1)(3)
    n, g = 40_000_000, 10_000_000
    off = rel.tuning(fanout=-1)
    single = L.rel_groupby_ws(1, k1, 2, aggs, n, g, ctypes.byref(off))
    part = L.rel_groupby_ws(1, k1, 2, aggs, n, g, None)
    assert part >= single + 2 * 16 * n
    # groups that fit the single pass's LDS table, or few rows: no buffers
    assert L.rel_groupby_ws(1, k1, 2, aggs, n, 100, None) == \
        L.rel_groupby_ws(1, k1, 2, aggs, n, 100, ctypes.byref(off))
    assert L.rel_groupby_ws(1, k1, 2, aggs, 500_000, 10_000, None) == \
        L.rel_groupby_ws(1, k1, 2, aggs, 500_000, 10_000, ctypes.byref(off))
    # groups beyond it over many rows: partitioned
    assert L.rel_groupby_ws(1, k1, 2, aggs, n, 10_000, None) >= 2 * 16 * n
    forced = rel.tuning(fanout=64)
    assert L.rel_groupby_ws(1, k1, 2, aggs, 1000, 100, ctypes.byref(forced)) >= 2 * 16 * 1000
    for bad in (3, 2, 100, 1 << 15, -2):
        t = rel.tuning(fanout=bad)
        assert L.rel_groupby_ws(1, k1, 2, aggs, 1000, 100, ctypes.byref(t)) == 0


def test_join_and_groupby_validation():
    L = rel.lib()
    b, p = col(100, 2), col(100, 3)
    rc = L.rel_hash_join(ctypes.byref(b), ctypes.byref(p), ctypes.c_void_p(1), ctypes.c_void_p(1),
                         10, ctypes.c_void_p(8), None, ctypes.c_void_p(0x10000), 1 << 30, None)
    assert rc == rel.REL_EINVAL and b"differ" in L.rel_last_error()
    bad_t = rel.tuning(load_factor=0.95)
    b = col(100, 2)
    p = col(100, 2)
    rc = L.rel_hash_join(ctypes.byref(b), ctypes.byref(p), ctypes.c_void_p(1), ctypes.c_void_p(1),
                         10, ctypes.c_void_p(8), ctypes.byref(bad_t), ctypes.c_void_p(0x10000),
                         1 << 30, None)
    assert rc == rel.REL_EINVAL
    keys = (rel.Column * 2)(col(50, 3), col(50, 2))
    vals = (rel.Column * 1)(col(50, 3))
    aggs = (rel.Agg * 1)(rel.Agg(0, 0))
    outs = (ctypes.c_void_p * 8)(*([0x100] * 8))
    rc = L.rel_groupby_agg(keys, 2, vals, 1, aggs, 1, outs, outs, 10, ctypes.c_void_p(8), 10,
                           None, ctypes.c_void_p(0x10000), 1 << 30, None)
    assert rc == rel.REL_EUNSUPPORTED
    aggs_bad = (rel.Agg * 1)(rel.Agg(0, 3))
    rc = L.rel_groupby_agg(keys, 1, vals, 1, aggs_bad, 1, outs, outs, 10, ctypes.c_void_p(8), 10,
                           None, ctypes.c_void_p(0x10000), 1 << 30, None)
    assert rc == rel.REL_EINVAL


def test_pipeline_validation():
    L = rel.lib()
    fact = (rel.Column * 2)(col(1000, 2), col(1000, 3, data=0x2000))
    preds = (rel.Pred * 1)(rel.Pred(0, 0, 5, 0))
    dims = (rel.Dim * 1)(rel.Dim(0, 1, col(30, 2, data=0x3000), col(30, 2, data=0x4000)))
    keys = (rel.KeyRef * 1)(rel.KeyRef(1, 0))
    aggs = (rel.Agg * 2)(rel.Agg(0, 1), rel.Agg(4, 1))

    def desc(**kw):
        d = rel.PipelineDesc(ctypes.cast(fact, ctypes.POINTER(rel.Column)), 2,
                             ctypes.cast(preds, ctypes.POINTER(rel.Pred)), 1,
                             ctypes.cast(dims, ctypes.POINTER(rel.Dim)), 1,
                             ctypes.cast(keys, ctypes.POINTER(rel.KeyRef)), 1,
                             ctypes.cast(aggs, ctypes.POINTER(rel.Agg)), 2, 64, None)
        for k, v in kw.items():
            setattr(d, k, v)
        return d

    good = desc()
    assert L.rel_pipeline_ws(ctypes.byref(good)) > 30 * 8
    assert L.rel_pipeline_ws(ctypes.byref(desc(n_dims=3))) == 0
    assert L.rel_pipeline_ws(ctypes.byref(desc(n_aggs=0))) == 0
    outs = rel.Outputs()
    rc = L.rel_pipeline(ctypes.byref(good), ctypes.byref(outs), ctypes.c_void_p(0x10000), 1 << 30, None)
    assert rc == rel.REL_EINVAL   # output pointers missing
    # a key naming a dim without payload
    dims[0].has_payload = 0
    assert L.rel_pipeline_ws(ctypes.byref(desc())) == 0
    dims[0].has_payload = 1
    # foreign keys of type int64 into int32 dim keys cannot match exactly
    dims[0].fact_col = 1
    assert L.rel_pipeline_ws(ctypes.byref(desc())) == 0


def test_binding_refuses_cpu_tensors():
    import torch
    with pytest.raises((RuntimeError, ValueError)):
        rel.filter([torch.zeros(10, dtype=torch.int32)], [(0, "lt", 3)])


def _batch_descs(n, dim_types, payloads, fact_len=1000, dim_len=30):
    keep = []
    descs = (rel.PipelineDesc * n)()
    for i in range(n):
        fact = (rel.Column * 2)(col(fact_len + i, 2), col(fact_len + i, 3, data=0x2000))
        dims = (rel.Dim * 1)(rel.Dim(0, payloads[i], col(dim_len * (i + 1), dim_types[i], data=0x3000),
                                     col(dim_len * (i + 1), 2, data=0x4000) if payloads[i]
                                     else rel.Column()))
        keys = (rel.KeyRef * 1)(rel.KeyRef(1, 0) if payloads[i] else rel.KeyRef(0, 0))
        aggs = (rel.Agg * 2)(rel.Agg(0, 1), rel.Agg(1, 0))
        keep += [fact, dims, keys, aggs]
        descs[i] = rel.PipelineDesc(ctypes.cast(fact, ctypes.POINTER(rel.Column)), 2, None, 0,
                                    ctypes.cast(dims, ctypes.POINTER(rel.Dim)), 1,
                                    ctypes.cast(keys, ctypes.POINTER(rel.KeyRef)), 1,
                                    ctypes.cast(aggs, ctypes.POINTER(rel.Agg)), 2, 64 * (i + 1),
                                    None)
    return descs, keep


def test_batch_validation_and_workspace():
    L = rel.lib()
    descs, keep = _batch_descs(3, [2, 2, 2], [1, 1, 1])
    total = L.rel_pipeline_batch_ws(descs, 3)
    # at least every plan's own tables
    assert total > sum(L.rel_pipeline_ws(ctypes.byref(descs[i])) for i in range(3)) // 2
    one = L.rel_pipeline_batch_ws(descs, 1)
    assert 0 < one < total
    assert L.rel_pipeline_batch_ws(descs, 0) == 0
    # plans must share a shape: dim key type, payload presence
    mixed, keep2 = _batch_descs(3, [2, 3, 2], [1, 1, 1])
    assert L.rel_pipeline_batch_ws(mixed, 3) == 0
    rc = L.rel_pipeline_batch(mixed, 3, None, None, 0, None)
    assert rc == rel.REL_EINVAL and b"differs" in L.rel_last_error()
    mixed, keep3 = _batch_descs(2, [2, 2], [1, 0])
    assert L.rel_pipeline_batch_ws(mixed, 2) == 0
    # outputs are required, and a short workspace is refused before any launch
    rc = L.rel_pipeline_batch(descs, 3, None, ctypes.c_void_p(0x10000), total, None)
    assert rc == rel.REL_EINVAL
    outs = (rel.Outputs * 3)()
    for o in outs:
        o.keys[0] = 0x100
        o.aggs[0] = 0x100
        o.aggs[1] = 0x100
        o.cap = 10
        o.d_groups = 0x200
    rc = L.rel_pipeline_batch(descs, 3, outs, ctypes.c_void_p(0x10000), total - 1, None)
    assert rc == rel.REL_ENOMEM
    g = ctypes.c_void_p()
    rc = L.rel_pipeline_batch_graph(descs, 3, outs, ctypes.c_void_p(0x10000), total - 1,
                                    ctypes.byref(g))
    assert rc == rel.REL_ENOMEM and not g.value
    assert L.rel_graph_launch(None, None) == rel.REL_EINVAL
    L.rel_graph_destroy(None)
    # chunk size is a tuning field that must not be negative
    t = rel.tuning(chunk_tiles=-1)
    descs[0].tuning = ctypes.pointer(t)
    assert L.rel_pipeline_batch_ws(descs, 3) == 0


def test_stream_read_validation():
    L = rel.lib()
    P = ctypes.c_void_p
    assert L.rel_stream_read(P(0x1000), -1, P(0x2000), None) == rel.REL_EINVAL
    assert L.rel_stream_read(P(0), 16, P(0x2000), None) == rel.REL_EINVAL
    assert L.rel_stream_read(P(0x1001), 16, P(0x2000), None) == rel.REL_EINVAL
    assert b"16-byte aligned" in L.rel_last_error()
    assert L.rel_stream_read(P(0x1000), 16, P(0), None) == rel.REL_EINVAL
    assert L.rel_stream_read(P(0x1000), 16, P(0x2004), None) == rel.REL_EINVAL
    assert L.rel_kernel_name(8) == b"stream_read"


def test_filter_noalloc_validation():
    L = rel.lib()
    P = ctypes.c_void_p
    ok_pred = (rel.Pred * 1)(rel.Pred(0, 0, 5, 0))

    def call(n, d_count=0x2000):
        ca = (rel.Column * 1)(col(n))
        return L.rel_filter_noalloc(ca, 1, ok_pred, 1, P(0x3000), n, P(d_count), None)

    assert call(10, d_count=0) == rel.REL_EINVAL
    # beyond the static scratch's 131040 tile states: rejected before any HIP call
    assert call(2_146_959_360 + 1) == rel.REL_ECAPACITY
    assert b"static scratch" in L.rel_last_error()


def test_bloom_validation_and_sizes():
    L = rel.lib()
    P = ctypes.c_void_p
    assert L.rel_bloom_bytes(0, 0) == 32
    assert L.rel_bloom_bytes(1000, 16) == 32 * 64  # 1000*16/256 = 62.5 -> 64 blocks
    assert L.rel_bloom_bytes(1000, 3) == 0 and L.rel_bloom_bytes(-1, 0) == 0
    c = rel.Column(0x1000, None, 100, 2, 0)
    assert L.rel_bloom_build(ctypes.byref(c), P(0x2010), 64, None) == rel.REL_EINVAL  # misaligned
    assert L.rel_bloom_build(ctypes.byref(c), P(0x2000), 96, None) == rel.REL_EINVAL  # 3 blocks
    assert L.rel_bloom_build(ctypes.byref(c), P(0), 64, None) == rel.REL_EINVAL
    need = L.rel_filter_ws(100)
    assert L.rel_bloom_filter(ctypes.byref(c), P(0x2000), 64, P(0x3000), 100, P(0x4000),
                              P(0x10000), need - 1, None) == rel.REL_ENOMEM
    assert L.rel_bloom_filter(ctypes.byref(c), P(0x2000), 64, P(0x3000), 100, P(0),
                              P(0x10000), need, None) == rel.REL_EINVAL
    plain = L.rel_hash_join_ws(3, 1_000_000, None)
    bloom = L.rel_hash_join_ws(3, 1_000_000, ctypes.byref(rel.tuning(flags=rel.TUNE_BLOOM)))
    assert bloom >= plain + L.rel_bloom_bytes(1_000_000, 16)
    t = rel.tuning(flags=8)
    assert L.rel_hash_join_ws(3, 1000, ctypes.byref(t)) == 0  # unknown flag bit


def test_gather_and_topn_validation():
    L = rel.lib()
    P = ctypes.c_void_p
    c = (rel.Column * 1)(rel.Column(0x1000, None, 100, 2, 0))
    outs = (ctypes.c_void_p * 1)(0x5000)
    assert L.rel_gather(c, 0, P(0x2000), 10, outs, None) == rel.REL_EINVAL
    assert L.rel_gather(c, 1, P(0), 10, outs, None) == rel.REL_EINVAL
    ci = (rel.Column * 1)(rel.Column(0x1000, 0x3000, 100, 2, 0))
    assert L.rel_gather(ci, 1, P(0x2000), 10, outs, None) == rel.REL_EINVAL
    assert L.rel_topn_ws(1000, 1025) == 0 and L.rel_topn_ws(1000, 10) > 0
    ws = L.rel_topn_ws(1000, 10)
    assert L.rel_topn(P(0x1000), 3, 1, None, 0, 1000, 1025, P(0x2000), P(0x3000), P(0x10000), ws,
                      None) == rel.REL_EINVAL
    assert L.rel_topn(P(0x1000), 2, 1, None, 0, 1000, 10, P(0x2000), P(0x3000), P(0x10000), ws,
                      None) == rel.REL_EINVAL  # int32 order column
    assert L.rel_topn(P(0x1004), 3, 1, None, 0, 1000, 10, P(0x2000), P(0x3000), P(0x10000), ws,
                      None) == rel.REL_EINVAL  # misaligned order
    assert L.rel_topn(P(0x1000), 4, 1, None, 0, 1000, 10, P(0x2000), P(0x3000), P(0x10000),
                      ws - 1, None) == rel.REL_ENOMEM
    short = (rel.Column * 1)(rel.Column(0x1000, None, 999, 3, 0))
    assert L.rel_topn(P(0x1000), 3, 1, short, 1, 1000, 10, P(0x2000), P(0x3000), P(0x10000), ws,
                      None) == rel.REL_EINVAL  # key shorter than the table


def test_binding_sizes_profile_arrays_like_the_header():
    """rel_profile_read writes REL_K_COUNT entries: the binding's arrays must
    be that long (a shorter one would be overwritten)."""
    text = open(HEADER).read()
    count = int(re.search(r"REL_K_COUNT\s*=\s*(\d+)", text).group(1))
    assert rel.KERNEL_CLASSES == count
    names = {rel.lib().rel_kernel_name(k).decode() for k in range(count)}
    assert "unknown" not in names and len(names) == count


def test_pipeline_stream_validation():
    L = rel.lib()
    P = ctypes.c_void_p
    fact = (rel.Column * 1)(rel.Column(0x1000, None, 10_000, 2, 0))
    aggs = (rel.Agg * 1)(rel.Agg(1, 0))
    d = rel.PipelineDesc(ctypes.cast(fact, ctypes.POINTER(rel.Column)), 1, None, 0, None, 0, None,
                         0, ctypes.cast(aggs, ctypes.POINTER(rel.Agg)), 1, 1, None)
    assert L.rel_pipeline_stream_ws(ctypes.byref(d), 1000) == 0  # not a multiple of 2048
    ws = L.rel_pipeline_stream_ws(ctypes.byref(d), 4096)
    assert ws >= L.rel_pipeline_ws(ctypes.byref(d)) + 2 * 4096 * 4
    o = rel.Outputs()
    o.aggs[0] = 0x5000
    o.cap = 1
    o.d_groups = 0x6000
    assert L.rel_pipeline_stream(ctypes.byref(d), 3000, ctypes.byref(o), P(0x10000), ws,
                                 None) == rel.REL_EINVAL
    assert L.rel_pipeline_stream(ctypes.byref(d), 4096, ctypes.byref(o), P(0x10000), ws - 1,
                                 None) == rel.REL_ENOMEM


def test_string_groupby_validation_and_workspace():
    L = rel.lib()
    P = ctypes.c_void_p
    aggs = (rel.Agg * 1)(rel.Agg(1, 0))
    assert L.rel_groupby_str_ws(100, -1, 1, aggs) == 0
    assert L.rel_groupby_str_ws(-1, 0, 1, aggs) == 0
    plain = L.rel_groupby_str_ws(100, 0, 1, aggs)
    dicted = L.rel_groupby_str_ws(100, 1000, 1, aggs)
    assert 0 < plain < dicted
    # the dictionary's string table (2 x 1000 claim words, rounded up to a
    # power of two) and one canonical id per entry
    assert dicted - plain >= 2048 * 8 + 1000 * 4
    vals = (rel.Column * 1)(rel.Column(0x1000, None, 500, 3, 0))
    cnt = P(0x9000)

    def call(st, ws_bytes):
        return L.rel_groupby_str(ctypes.byref(st), None, vals, 1, aggs, 1, P(0x2000), None,
                                 (P * 1)(0x3000), 100, cnt, 100, P(0x10000), ws_bytes, None)

    coded = rel.Strings(0x4000, 0x5000, 0x6000, 500, 1000)
    # a workspace sized without the dictionary is too small for its codes
    assert call(coded, plain) == rel.REL_ENOMEM
    assert call(rel.Strings(0x4000, 0x5000, None, 500, 1000), plain) == rel.REL_EINVAL


def _group_plan(fact_len, max_groups, t=None):
    """One join + group-by description (int32 foreign keys into a 1000-key
    dim with an int32 payload as the group key, SUM of an int64 column and
    COUNT) over fake device addresses: workspace sizing reads no data."""
    fact = (rel.Column * 2)(col(fact_len, 2), col(fact_len, 3, data=0x2000))
    dims = (rel.Dim * 1)(rel.Dim(0, 1, col(1000, 2, data=0x3000), col(1000, 2, data=0x4000)))
    keys = (rel.KeyRef * 1)(rel.KeyRef(1, 0))
    aggs = (rel.Agg * 2)(rel.Agg(0, 1), rel.Agg(1, 0))
    d = rel.PipelineDesc(ctypes.cast(fact, ctypes.POINTER(rel.Column)), 2, None, 0,
                         ctypes.cast(dims, ctypes.POINTER(rel.Dim)), 1,
                         ctypes.cast(keys, ctypes.POINTER(rel.KeyRef)), 1,
                         ctypes.cast(aggs, ctypes.POINTER(rel.Agg)), 2, max_groups,
                         ctypes.pointer(t) if t is not None else None)
    return d, [fact, dims, keys, aggs, t]


def test_batch_record_workspace():
    """A batched plan whose groups outgrow the LDS table takes two record
    regions of 12 bytes a row (32-bit keys, one value column): the fused
    pass's runs and the partitioned copy. tuning.fanout -1 takes none, and
    records stop once a batch's regions would pass 64 GiB."""
    L = rel.lib()
    rows = 10_000_000
    d, keep = _group_plan(rows, 100_000)
    off_t = rel.tuning(fanout=-1)
    d_off, keep2 = _group_plan(rows, 100_000, off_t)
    with_rec = L.rel_pipeline_batch_ws(ctypes.byref(d), 1)
    without = L.rel_pipeline_batch_ws(ctypes.byref(d_off), 1)
    assert with_rec > 0 and without > 0
    extra = with_rec - without
    assert 2 * rows * 12 <= extra <= 2 * rows * 12 + (64 << 20), extra
    # few groups: the LDS table holds them, no records
    small, keep3 = _group_plan(rows, 100)
    small_off, keep4 = _group_plan(rows, 100, off_t)
    assert L.rel_pipeline_batch_ws(ctypes.byref(small), 1) == \
        L.rel_pipeline_batch_ws(ctypes.byref(small_off), 1)
    # the 64 GiB bound: a 2^31-row plan's records (about 51.5 GB) fit once
    big = 1 << 31
    descs = (rel.PipelineDesc * 2)()
    b0, k0 = _group_plan(big, 100_000)
    b1, k1 = _group_plan(big, 100_000)
    descs[0], descs[1] = b0, b1
    one = L.rel_pipeline_batch_ws(descs, 1)
    two = L.rel_pipeline_batch_ws(descs, 2)
    assert one > 2 * big * 12
    assert two - one < 2 * big * 12  # the second plan keeps the atomics
