"""Hash group-by on string keys (rel_groupby_str) against the oracle: plain
and dictionary-encoded columns (a dictionary holding the same string under
several codes must still give one group), an integer key beside the string,
empty strings, strings longer than a wave's worth of words, every start
alignment of the byte offsets, heavy skew (hot keys pre-aggregated in LDS,
the rest straight to the global table) and the group bound; groups compared after sorting by (string, integer key), with
the smallest row id of each group exact."""

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import announce, dev
from paper_2508_04701_amd import rel

pytestmark = pytest.mark.gpu

AGGS = [("sum", 0), ("count", None), ("min", 1), ("max", 1), ("avg", 0)]


def make_strings(r, nstr, maxlen, alphabet=26):
    lens = r.integers(0, maxlen + 1, size=nstr)
    data = r.integers(97, 97 + alphabet, size=int(lens.sum())).astype(np.uint8)
    offsets = np.zeros(nstr + 1, np.int64)
    offsets[1:] = np.cumsum(lens)
    return offsets, data


def expand(offsets, data, codes):
    """The materialised strings of a dictionary-encoded column (for the oracle)."""
    parts = [data[offsets[c]:offsets[c + 1]] for c in codes]
    lens = np.array([len(x) for x in parts], np.int64)
    off = np.zeros(len(codes) + 1, np.int64)
    off[1:] = np.cumsum(lens)
    return off, (np.concatenate(parts) if parts and off[-1] else np.zeros(0, np.uint8))


def check(got, want, aggs, what):
    rows, iks, ga = got
    wr, wik, wa = want
    rows = rows.cpu().numpy().view(np.uint32)
    assert len(rows) == len(wr), f"{what}: {len(rows)} groups, oracle {len(wr)}"
    # match groups by their first row (unique per group)
    order = np.argsort(rows)
    wo = np.argsort(wr)
    assert np.array_equal(rows[order], wr[wo]), f"{what}: first rows differ"
    if iks is not None:
        assert np.array_equal(iks.cpu().numpy().astype(np.int64)[order], wik[wo]), f"{what}: int keys"
    for a, (op, _) in enumerate(aggs):
        g = ga[a].cpu().numpy().view(np.int64)[order]
        w = np.asarray(wa[a]).view(np.int64)[wo]
        assert np.array_equal(g, w), f"{what}: {op}"


@pytest.mark.parametrize("n,nstr,maxlen", [(1, 1, 0), (1000, 50, 3), (100_003, 5000, 40),
                                           (400_000, 100_000, 90)])
def test_string_groupby_plain(n, nstr, maxlen):
    announce("string group-by plain", n, nstr, maxlen)
    r = np.random.default_rng(n + maxlen)
    d_off, d_data = make_strings(r, nstr, maxlen, alphabet=4 if maxlen < 10 else 26)
    codes = r.integers(0, nstr, size=n)
    off, data = expand(d_off, d_data, codes)
    v0 = r.integers(-10**9, 10**9, size=n).astype(np.int64)
    v1 = r.integers(-1000, 1000, size=n).astype(np.int32)
    got = rel.groupby_str(dev(off), dev(data), [dev(v0), dev(v1)], AGGS)
    want = oracle.groupby_str(off, data, [v0, v1], AGGS)
    check(got, want, AGGS, f"plain n={n}")


def test_string_groupby_dictionary_with_duplicate_entries_and_int_key():
    announce("string group-by dictionary")
    r = np.random.default_rng(4)
    d_off, d_data = make_strings(r, 3000, 12, alphabet=3)  # many repeated strings
    n = 300_000
    codes = r.integers(0, 3000, size=n).astype(np.int32)
    ikey = r.integers(-2, 2, size=n).astype(np.int8)
    v0 = r.integers(0, 10**6, size=n).astype(np.int64)
    v1 = r.integers(0, 100, size=n).astype(np.int64)
    got = rel.groupby_str(dev(d_off), dev(d_data), [dev(v0), dev(v1)], AGGS, ikey=dev(ikey),
                          codes=dev(codes))
    off, data = expand(d_off, d_data, codes)
    want = oracle.groupby_str(off, data, [v0, v1], AGGS, ikey=ikey)
    check(got, want, AGGS, "dictionary + int key")


def test_string_groupby_skew_and_alignment():
    """Zipf-like skew (a few strings hold most rows) over strings starting at
    every byte alignment."""
    announce("string group-by skew")
    r = np.random.default_rng(5)
    d_off, d_data = make_strings(r, 20_000, 33)
    n = 1_000_000
    hot = (r.pareto(1.2, size=n) * 3).astype(np.int64) % 20_000
    off, data = expand(d_off, d_data, hot)
    v0 = r.integers(0, 10**6, size=n).astype(np.int64)
    v1 = r.integers(-5, 5, size=n).astype(np.int64)
    got = rel.groupby_str(dev(off), dev(data), [dev(v0), dev(v1)], AGGS, max_groups=20_000)
    want = oracle.groupby_str(off, data, [v0, v1], AGGS)
    check(got, want, AGGS, "skew")


def test_string_groupby_too_many_groups():
    announce("string group-by bound")
    r = np.random.default_rng(6)
    off, data = make_strings(r, 5000, 20)
    v = np.arange(5000, dtype=np.int64)
    with pytest.raises(rel.RelError) as e:
        rel.groupby_str(dev(off), dev(data), [dev(v)], [("count", None)], max_groups=10)
    assert e.value.status == rel.REL_ECAPACITY


def test_string_groupby_dictionary_zipf_many_groups():
    """Dictionary codes drawn by Zipf rank over 60k entries that repeat
    strings: more distinct slots than a workgroup's LDS table holds, so rows
    take both the LDS and the global update path."""
    announce("string group-by dictionary zipf")
    r = np.random.default_rng(7)
    d_off, d_data = make_strings(r, 60_000, 7, alphabet=5)
    n = 2_000_000
    codes = (np.minimum(r.zipf(1.1, size=n), 60_000) - 1).astype(np.int32)
    v0 = r.integers(-10**9, 10**9, size=n).astype(np.int64)
    v1 = r.integers(-1000, 1000, size=n).astype(np.int64)
    got = rel.groupby_str(dev(d_off), dev(d_data), [dev(v0), dev(v1)], AGGS, codes=dev(codes))
    off, data = expand(d_off, d_data, codes)
    want = oracle.groupby_str(off, data, [v0, v1], AGGS)
    check(got, want, AGGS, "dictionary zipf")


def test_string_groupby_dictionary_too_many_groups():
    announce("string group-by dictionary bound")
    r = np.random.default_rng(8)
    off, data = make_strings(r, 5000, 20)
    codes = np.arange(5000, dtype=np.int32)[::-1].copy()
    v = np.arange(5000, dtype=np.int64)
    with pytest.raises(rel.RelError) as e:
        rel.groupby_str(dev(off), dev(data), [dev(v)], [("count", None)], codes=dev(codes),
                        max_groups=10)
    assert e.value.status == rel.REL_ECAPACITY
