"""Checks that pin the oracle to facts other than itself.

Each ``pin_*`` function takes an ``oracle.Oracle`` and raises AssertionError
when the oracle disagrees with:
  * brute force on tiny inputs (nested-loop join, sort-and-scan group-by,
    a plain loop for the filter), written without hash maps;
  * closed forms on designed inputs;
  * invariants that hold at any size (|join| = sum_k bc(k) * pc(k),
    sum COUNT = rows entering the group-by, sum SUM = total SUM mod 2^64,
    global MIN/MAX, MIN <= AVG <= MAX);
  * special cases that reduce to a library routine.
``tests/test_oracle_pins.py`` runs them against the oracle;
``tests/test_oracle_mutants.py`` runs them against deliberately broken builds
of the oracle and expects each build to be caught.
"""

from __future__ import annotations

import operator
from fractions import Fraction

import numpy as np

I64_MIN, I64_MAX = -(2**63), 2**63 - 1
I32_MIN, I32_MAX = -(2**31), 2**31 - 1
NAN_BITS = 0x7FF8000000000000

_CMP = {
    "lt": lambda v, lo, hi: operator.lt(v, lo),
    "le": lambda v, lo, hi: operator.le(v, lo),
    "gt": lambda v, lo, hi: operator.gt(v, lo),
    "ge": lambda v, lo, hi: operator.ge(v, lo),
    "eq": lambda v, lo, hi: operator.eq(v, lo),
    "ne": lambda v, lo, hi: operator.ne(v, lo),
    "range": lambda v, lo, hi: lo <= v and v < hi,
}
_NEGATE = {"lt": "ge", "ge": "lt", "le": "gt", "gt": "le", "eq": "ne", "ne": "eq"}


def wrap64(x: int) -> int:
    """Two's-complement int64 value of the integer x (mod 2^64)."""
    return (x + 2**63) % 2**64 - 2**63


def avg_value(s: int, c: int) -> float:
    """Binary64 AVG of an exact int64 SUM and COUNT. Below 2^53 the int64 to
    double conversion is exact, so the result is the correctly rounded
    quotient, computed here from the exact rational."""
    if c == 0:
        return np.frombuffer(np.int64(NAN_BITS).tobytes(), dtype=np.float64)[0]
    if abs(s) < 2**53:
        return float(Fraction(s, c))
    return float(s) / float(c)


# ------------------------------------------------------------------ brute force

def bf_filter(cols, terms, sel=None):
    rows = range(len(cols[0])) if sel is None else [int(r) for r in sel]
    out = []
    for r in rows:
        if all(_CMP[op](int(cols[c][r]), lo, (t[3] if len(t) > 3 else None))
               for t in terms for (c, op, lo) in [t[:3]]):
            out.append(r)
    return np.array(out, dtype=np.uint32)


def bf_join(build, probe):
    pairs = [(b, p) for p in range(len(probe)) for b in range(len(build)) if build[b] == probe[p]]
    ob = np.array([b for b, _ in pairs], dtype=np.uint32)
    op = np.array([p for _, p in pairs], dtype=np.uint32)
    return ob, op


def bf_group_rows(rows, aggs):
    """rows: list of (key tuple, [value per agg]). Sort by key, scan runs."""
    rows = sorted(rows, key=lambda r: r[0])
    keys, out = [], [[] for _ in aggs]
    i = 0
    while i < len(rows):
        j = i
        while j < len(rows) and rows[j][0] == rows[i][0]:
            j += 1
        keys.append(rows[i][0])
        run = rows[i:j]
        for a, (op, _) in enumerate(aggs):
            vs = [r[1][a] for r in run]
            if op == "sum":
                out[a].append(wrap64(sum(vs)))
            elif op == "count":
                out[a].append(len(vs))
            elif op == "min":
                out[a].append(min(vs))
            elif op == "max":
                out[a].append(max(vs))
            else:
                out[a].append(avg_value(wrap64(sum(vs)), len(vs)))
        i = j
    return keys, out


def bf_groupby(keys, vals, aggs):
    n = len(keys[0]) if keys else len(vals[0])
    rows = [(tuple(int(k[i]) for k in keys),
             [0 if op == "count" else int(vals[c][i]) for op, c in aggs]) for i in range(n)]
    return bf_group_rows(rows, aggs)


def bf_pipeline(fact, terms, dims, keys, aggs):
    n = len(fact[0])
    rows = []
    passing = set(int(r) for r in bf_filter(fact, terms))
    for i in range(n):
        if i not in passing:
            continue
        choices = [[None]]
        for d in dims:
            fk = int(fact[d["fk"]][i])
            choices.append([b for b in range(len(d["key"])) if int(d["key"][b]) == fk])
        combos = [[]]
        for ch in choices[1:]:
            combos = [c + [b] for c in combos for b in ch]
        for combo in combos:
            key = []
            for src, col in keys:
                if src == "fact":
                    key.append(int(fact[col][i]))
                else:
                    key.append(int(dims[col]["payload"][combo[col]]))
            rows.append((tuple(key), [0 if op == "count" else int(fact[c][i]) for op, c in aggs]))
    return bf_group_rows(rows, aggs)


# ------------------------------------------------------------------ comparisons

def assert_groups_equal(got, want, aggs, what=""):
    gk, ga = got
    wk, wa = want
    ng = len(wa[0]) if wa else len(wk)
    got_keys = list(zip(*[list(map(int, k)) for k in gk])) if gk else [()] * len(ga[0])
    assert len(got_keys) == ng, f"{what}: {len(got_keys)} groups, expected {ng}"
    assert [tuple(k) for k in got_keys] == [tuple(k) for k in wk], f"{what}: group keys differ"
    for a, (op, _) in enumerate(aggs):
        g = np.asarray(ga[a])
        w = wa[a]
        if op == "avg":
            gb = g.view(np.int64).tolist()
            wb = np.asarray(w, dtype=np.float64).view(np.int64).tolist()
            assert gb == wb, f"{what}: AVG bits differ"
        else:
            assert [int(x) for x in g] == [int(x) for x in w], f"{what}: {op} differs"


def assert_pairs_equal(got, want, what=""):
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), f"{what}: pairs differ"


# ------------------------------------------------------------------ pins

def _rng(seed):
    return np.random.default_rng(seed)


def _tiny_col(rng, n, dtype, domain):
    extremes = {np.int8: [-128, 127, -1, 0], np.int32: [I32_MIN, I32_MAX, -1, 0],
                np.int64: [I64_MIN, I64_MAX, -1, 0]}[dtype]
    vals = rng.integers(-domain, domain, size=n)
    pick = rng.random(n) < 0.15
    vals[pick] = rng.choice(extremes, size=int(pick.sum()))
    return vals.astype(dtype)


def pin_filter_brute_force(orc):
    for seed in range(12):
        rng = _rng(seed)
        n = int(rng.integers(0, 200))
        cols = [_tiny_col(rng, n, t, 6) for t in (np.int8, np.int32, np.int64)]
        terms = []
        for _ in range(int(rng.integers(1, 5))):
            op = str(rng.choice(list(_CMP)))
            c = int(rng.integers(0, 3))
            lo = int(rng.integers(-6, 6))
            hi = lo + int(rng.integers(0, 6))
            terms.append((c, op, lo, hi))
        sel = None
        if seed % 3 == 0 and n:
            sel = np.sort(rng.choice(n, size=n // 2, replace=False)).astype(np.uint32)
        got = orc.filter(cols, terms, sel)
        want = bf_filter(cols, terms, sel)
        assert np.array_equal(got, want), f"filter seed {seed}"


def pin_filter_closed_forms(orc):
    n = 100_003
    date = (np.arange(n) % 2557).astype(np.int32)
    for T in (0, 1, 767, 2556, 2557, 5000):
        got = orc.filter([date], [(0, "lt", T)])
        expect = (n // 2557) * min(T, 2557) + min(n % 2557, T)
        assert len(got) == expect, f"date < {T}: count"
        assert np.array_equal(got, np.flatnonzero(date < T).astype(np.uint32)), f"date < {T}: rows"
    always = orc.filter([date], [(0, "range", I64_MIN, I64_MAX)])
    assert np.array_equal(always, np.arange(n, dtype=np.uint32)), "always-true filter is iota"
    assert len(orc.filter([date], [(0, "range", 5, 5)])) == 0, "empty range selects nothing"
    # filter(P) and filter(not P) split the rows
    rng = _rng(7)
    x = rng.integers(-50, 50, size=5000).astype(np.int64)
    for op in _NEGATE:
        a = orc.filter([x], [(0, op, 3)])
        b = orc.filter([x], [(0, _NEGATE[op], 3)])
        assert np.all(np.diff(a.astype(np.int64)) > 0), "filter output strictly increasing"
        assert len(np.intersect1d(a, b)) == 0 and len(a) + len(b) == len(x), f"{op} partition"


def pin_join_brute_force(orc):
    for seed in range(12):
        rng = _rng(100 + seed)
        dtype = np.int32 if seed % 2 else np.int64
        nb, npr = int(rng.integers(0, 120)), int(rng.integers(0, 160))
        build = _tiny_col(rng, nb, dtype, 8)
        probe = _tiny_col(rng, npr, dtype, 8)
        assert_pairs_equal(orc.hash_join(build, probe), bf_join(build, probe), f"join seed {seed}")


def pin_join_closed_forms(orc):
    for n, m in ((0, 5), (7, 0), (1000, 700), (513, 4097)):
        b, p = orc.hash_join(np.arange(n, dtype=np.int32), np.arange(m, dtype=np.int32))
        k = min(n, m)
        assert np.array_equal(b, np.arange(k, dtype=np.uint32)) and np.array_equal(p, b), "iota join"
    for nb, npr, K in ((1000, 10_000, 1500), (1000, 9_999, 700), (64, 1000, 64)):
        b, p = orc.hash_join(np.arange(nb, dtype=np.int64), (np.arange(npr) % K).astype(np.int64))
        expect = (npr // K) * min(nb, K) + min(npr % K, nb)
        assert len(b) == expect, "p mod K join count"
        assert np.array_equal(b.astype(np.int64), p.astype(np.int64) % K), "p mod K pairs"


def pin_join_invariants(orc):
    rng = _rng(5)
    build = rng.integers(0, 3000, size=20_000).astype(np.int32)  # duplicates on both sides
    probe = rng.integers(0, 4000, size=50_000).astype(np.int32)
    b, p = orc.hash_join(build, probe)
    ub, cb = np.unique(build, return_counts=True)
    up, cp = np.unique(probe, return_counts=True)
    common, ib, ip = np.intersect1d(ub, up, return_indices=True)
    assert len(b) == int(np.sum(cb[ib].astype(np.int64) * cp[ip])), "|J| = sum bc*pc"
    assert b.max(initial=0) < len(build) and p.max(initial=0) < len(probe), "row ids in range"
    assert np.array_equal(build[b], probe[p]), "every pair matches"
    packed = p.astype(np.uint64) << np.uint64(32) | b.astype(np.uint64)
    assert len(packed) < 2 or np.all(packed[1:] > packed[:-1]), \
        "pairs sorted by (probe, build), no duplicates"


def pin_groupby_brute_force(orc):
    all_aggs = [("sum", 0), ("count", None), ("min", 1), ("max", 2), ("avg", 0), ("avg", 2)]
    for seed in range(12):
        rng = _rng(200 + seed)
        n = int(rng.integers(0, 200))
        nk = int(rng.integers(0, 3))
        ktypes = [np.int8, np.int32, np.int64]
        keys = [_tiny_col(rng, n, ktypes[int(rng.integers(0, 3))], 3) for _ in range(nk)]
        vals = [_tiny_col(rng, n, np.int64, 1000), _tiny_col(rng, n, np.int32, 50),
                _tiny_col(rng, n, np.int8, 20)]
        got = orc.groupby(keys, vals, all_aggs)
        if nk == 0:
            rows = [((), [0 if op == "count" else int(vals[c][i]) for op, c in all_aggs])
                    for i in range(n)]
            want = bf_group_rows(rows, all_aggs)
            if n == 0:
                want = ([()], [[0], [0], [I64_MAX], [I64_MIN], [avg_value(0, 0)], [avg_value(0, 0)]])
        else:
            want = bf_groupby(keys, vals, all_aggs)
        assert_groups_equal(got, want, all_aggs, f"groupby seed {seed}")


def pin_groupby_closed_forms(orc):
    n, G = 100_000, 37
    key = (np.arange(n) % G).astype(np.int32)
    v = np.arange(n, dtype=np.int64)
    aggs = [("count", None), ("sum", 0), ("min", 0), ("max", 0)]
    (k,), (cnt, s, mn, mx) = orc.groupby([key], [v], aggs)
    g = np.arange(G)
    c = (n - g + G - 1) // G
    assert np.array_equal(k, g), "keys 0..G-1"
    assert np.array_equal(cnt, c), "COUNT_g = ceil((n - g) / G)"
    assert np.array_equal(s, c * g + G * c * (c - 1) // 2), "SUM_g closed form"
    assert np.array_equal(mn, g) and np.array_equal(mx, g + (c - 1) * G), "MIN/MAX closed form"
    # all keys equal: one group equal to the plain reductions
    rng = _rng(9)
    x = rng.integers(-10**12, 10**12, size=10_000)
    (k1,), (s1, c1, lo1, hi1) = orc.groupby([np.full(10_000, -7, np.int64)], [x],
                                            [("sum", 0), ("count", None), ("min", 0), ("max", 0)])
    assert list(k1) == [-7] and int(s1[0]) == int(x.sum()) and int(c1[0]) == 10_000
    assert int(lo1[0]) == int(x.min()) and int(hi1[0]) == int(x.max()), "single group reductions"
    # all keys distinct: each group is its row
    perm = rng.permutation(5000).astype(np.int64) * 3 - 7000
    y = rng.integers(-100, 100, size=5000)
    (kd,), (sd, cd) = orc.groupby([perm], [y], [("sum", 0), ("count", None)])
    order = np.argsort(perm)
    assert np.array_equal(kd, perm[order]) and np.array_equal(sd, y[order]) and np.all(cd == 1)
    # grouped empty input: no groups; ungrouped empty input: one row, NaN AVG
    kk, aa = orc.groupby([np.zeros(0, np.int32)], [np.zeros(0, np.int64)], [("sum", 0), ("avg", 0)])
    assert len(kk[0]) == 0 and len(aa[0]) == 0, "grouped empty -> 0 groups"
    kk, aa = orc.groupby([], [np.zeros(0, np.int64)],
                         [("sum", 0), ("count", None), ("min", 0), ("max", 0), ("avg", 0)])
    assert all(len(a) == 1 for a in aa), "ungrouped empty input still yields one row"
    assert [int(a[0]) for a in aa[:4]] == [0, 0, I64_MAX, I64_MIN], "ungrouped empty"
    assert int(aa[4].view(np.int64)[0]) == NAN_BITS, "AVG over no rows is the canonical NaN"


def pin_groupby_arithmetic(orc):
    # SUM wraps modulo 2^64; AVG is the correctly rounded quotient below 2^53
    big = np.array([I64_MAX, 5, I64_MAX, I64_MIN, -3], dtype=np.int64)
    _, (s,) = orc.groupby([np.zeros(5, np.int32)], [big], [("sum", 0)])
    assert int(s[0]) == wrap64(sum(int(v) for v in big)), "SUM wraps mod 2^64"
    rng = _rng(11)
    for _ in range(5):
        n = int(rng.integers(1, 60))
        v = rng.integers(-(2**40), 2**40, size=n)
        _, (a,) = orc.groupby([np.zeros(n, np.int8)], [v], [("avg", 0)])
        assert float(a[0]) == float(Fraction(int(v.sum()), n)), "AVG correctly rounded"
    # AVG of 1, 2 (=1.5) and of 1, 1, 2 (=4/3, inexact) against exact rationals
    _, (a2,) = orc.groupby([np.zeros(3, np.int32)], [np.array([1, 1, 2], np.int64)], [("avg", 0)])
    assert float(a2[0]) == float(Fraction(4, 3))


def pin_pipeline_brute_force(orc):
    for seed in range(10):
        rng = _rng(300 + seed)
        n = int(rng.integers(0, 150))
        nd = int(rng.integers(0, 3))
        fact = [rng.integers(0, 12, size=n).astype(np.int32),     # fk 0
                rng.integers(-2, 9, size=n).astype(np.int64),     # fk 1
                rng.integers(0, 30, size=n).astype(np.int32),     # date
                _tiny_col(rng, n, np.int64, 10**6),               # price
                rng.integers(0, 3, size=n).astype(np.int8)]       # flag
        dims = []
        for d in range(nd):
            m = int(rng.integers(0, 14))
            dt = np.int32 if d == 0 else np.int64
            dims.append(dict(fk=d, key=rng.integers(-1, 12, size=m).astype(dt),  # dup keys possible
                             payload=rng.integers(-3, 4, size=m).astype(np.int32)))
        keys = [("fact", 4)] + [("dim", d) for d in range(nd)][:1]
        if seed % 4 == 3:
            keys = []
        aggs = [("sum", 3), ("count", None), ("avg", 3), ("min", 3), ("max", 3)]
        terms = [(2, "lt", int(rng.integers(0, 31)))]
        got = orc.pipeline(fact, terms, dims, keys, aggs)
        want = bf_pipeline(fact, terms, dims, keys, aggs)
        if not keys and not want[1][0]:
            want = ([()], [[0], [0], [avg_value(0, 0)], [I64_MAX], [I64_MIN]])
        assert_groups_equal(got, want, aggs, f"pipeline seed {seed}")


def pin_pipeline_invariants(orc):
    """Star-schema-shaped input: dims are FK-complete, so the rows entering
    the group-by are exactly the filtered rows."""
    rng = _rng(17)
    n, na, nb = 40_000, 3000, 200
    fk_a = rng.integers(0, na, size=n).astype(np.int32)
    fk_b = rng.integers(0, nb, size=n).astype(np.int32)
    date = rng.integers(0, 2557, size=n).astype(np.int32)
    price = rng.integers(100, 10**7, size=n).astype(np.int64)
    flag = rng.integers(0, 3, size=n).astype(np.int8)
    a_key = rng.permutation(na).astype(np.int32)
    b_key = rng.permutation(nb).astype(np.int32)
    region = rng.integers(0, 25, size=nb).astype(np.int32)
    fact = [fk_a, fk_b, date, price, flag]
    dims = [dict(fk=0, key=a_key, payload=None), dict(fk=1, key=b_key, payload=region)]
    aggs = [("sum", 3), ("count", None), ("avg", 3), ("min", 3), ("max", 3)]
    (kr, kf), (s, c, a, mn, mx) = orc.pipeline(fact, [(2, "lt", 767)], dims,
                                               [("dim", 1), ("fact", 4)], aggs)
    sel = date < 767
    assert int(c.sum()) == int(sel.sum()), "sum COUNT = filtered rows"
    assert int(s.sum()) == int(price[sel].sum()), "sum SUM = total SUM"
    assert int(mn.min()) == int(price[sel].min()) and int(mx.max()) == int(price[sel].max())
    assert np.all(c >= 1) and np.all(mn <= a) and np.all(a <= mx), "MIN <= AVG <= MAX"
    # marginals: per flag via a 3-bucket loop; per region via an array lookup of dim B
    region_of_fk = np.empty(nb, np.int64)
    region_of_fk[b_key] = region
    r = region_of_fk[fk_b]
    for f in range(3):
        m = sel & (flag == f)
        assert int(s[kf == f].sum()) == int(price[m].sum()), "flag marginal"
    for g in range(25):
        m = sel & (r == g)
        assert int(c[kr == g].sum()) == int(m.sum()), "region marginal"


# ------------------------------------------------------------- semi-join

def bf_semi_join(build, probe):
    """Nested loop: probe rows with at least one equal build key."""
    bl = [int(x) for x in build]
    return np.array([p for p, k in enumerate(int(x) for x in probe) if any(k == b for b in bl)],
                    dtype=np.uint32)


def pin_semi_join_brute_force(orc):
    for seed in range(12):
        rng = _rng(400 + seed)
        dtype = np.int32 if seed % 2 else np.int64
        build = _tiny_col(rng, int(rng.integers(0, 100)), dtype, 8)
        probe = _tiny_col(rng, int(rng.integers(0, 150)), dtype, 10)
        assert np.array_equal(orc.semi_join(build, probe), bf_semi_join(build, probe)), \
            f"semi-join seed {seed}"


def pin_semi_join_closed_forms(orc):
    # build = iota(nb), probe p = p mod K: p matches iff p mod K < nb
    for nb, npr, K in ((1000, 10_000, 1500), (64, 5000, 64), (0, 100, 7), (10, 0, 3)):
        got = orc.semi_join(np.arange(nb, dtype=np.int64), (np.arange(npr) % K).astype(np.int64))
        expect = (npr // K) * min(nb, K) + min(npr % K, nb) if K else 0
        assert len(got) == expect, "semi-join count"
        assert np.all(got % K < nb) and np.all(np.diff(got.astype(np.int64)) > 0), "rows, order"
    # duplicates on the build side do not repeat probe rows
    b = np.array([5, 5, 5, 7], np.int32)
    p = np.array([7, 5, 1, 5], np.int32)
    assert np.array_equal(orc.semi_join(b, p), np.array([0, 1, 3], np.uint32)), "dup build keys"


# --------------------------------------------------------------- gather

def pin_gather(orc):
    rng = _rng(8)
    for dtype in (np.int8, np.int32, np.int64):
        col = _tiny_col(rng, 500, dtype, 1000)
        idx = rng.integers(0, 500, size=2000).astype(np.uint32)
        got = orc.gather(col, idx)
        assert got.dtype == np.int64
        assert np.array_equal(got, col[idx].astype(np.int64)), f"gather {dtype}"  # numpy indexing
    assert len(orc.gather(np.zeros(3, np.int32), np.zeros(0, np.uint32))) == 0


# ---------------------------------------------------------------- top-N

def _check_topn(order, keys, limit, desc, got):
    """Selection property, without sorting: the result is ordered, and no
    left-out row comes before the last one taken (order value, then key tuple)."""
    n = len(order)
    assert len(got) == min(limit, n), "top-N size"
    assert len(set(got.tolist())) == len(got), "top-N rows distinct"

    def before(a, b):
        x, y = order[a], order[b]
        if x != y:
            return x > y if desc else x < y
        return tuple(int(k[a]) for k in keys) < tuple(int(k[b]) for k in keys)

    for i in range(1, len(got)):
        assert before(got[i - 1], got[i]), "top-N ordered"
    if len(got) and len(got) < n:
        last = got[-1]
        left = set(range(n)) - set(got.tolist())
        assert not any(before(r, last) for r in left), "a left-out row belongs in the top-N"


def pin_topn_selection(orc):
    for seed in range(10):
        rng = _rng(500 + seed)
        n = int(rng.integers(0, 300))
        keys = [rng.permutation(n).astype(np.int64)] if seed % 2 else \
            [rng.integers(0, 5, size=n).astype(np.int64), rng.permutation(n).astype(np.int64)]
        if seed % 3 == 0:
            order = rng.normal(size=n).round(1)  # float64 with ties
        else:
            order = rng.integers(-5, 5, size=n).astype(np.int64)  # heavy ties
        for limit in (0, 1, 7, n, n + 5):
            for desc in (True, False):
                _check_topn(order, keys, limit, desc, orc.topn(order, keys, limit, desc))
    # all values distinct: the top-N of a permutation is closed-form
    perm = _rng(9).permutation(1000).astype(np.int64)
    got = orc.topn(perm, [np.arange(1000, dtype=np.int64)], 10)
    assert np.array_equal(perm[got], np.arange(999, 989, -1)), "top-10 of a permutation"


# ------------------------------------------------------ string group-by

def _strings(rng, n, alphabet=3, maxlen=4):
    words = ["".join(chr(97 + int(c)) for c in rng.integers(0, alphabet, size=int(rng.integers(0, maxlen + 1))))
             for _ in range(n)]
    data = "".join(words).encode()
    offsets = np.zeros(n + 1, np.int64)
    offsets[1:] = np.cumsum([len(w) for w in words])
    return words, offsets, np.frombuffer(data, dtype=np.uint8).copy() if data else np.zeros(0, np.uint8)


def pin_groupby_str_brute_force(orc):
    aggs = [("sum", 0), ("count", None), ("min", 0), ("max", 0), ("avg", 0)]
    for seed in range(10):
        rng = _rng(600 + seed)
        n = int(rng.integers(0, 150))
        words, offsets, data = _strings(rng, n)
        v = _tiny_col(rng, n, np.int64, 1000)
        ik = rng.integers(-2, 2, size=n).astype(np.int32) if seed % 2 else None
        rows, iks, got = orc.groupby_str(offsets, data, [v], aggs, ik)
        # brute force: a dict keyed by (bytes, int key), ordered by sorting
        groups = {}
        for i, w in enumerate(words):
            key = (w.encode(), int(ik[i]) if ik is not None else 0)
            groups.setdefault(key, []).append(i)
        order = sorted(groups)
        assert len(rows) == len(order), f"string groups seed {seed}"
        for g, key in enumerate(order):
            members = groups[key]
            assert rows[g] == members[0] and iks[g] == key[1], "first row and int key"
            vals = [int(v[i]) for i in members]
            assert got[0][g] == wrap64(sum(vals)) and got[1][g] == len(vals)
            assert got[2][g] == min(vals) and got[3][g] == max(vals)
            assert got[4][g] == avg_value(wrap64(sum(vals)), len(vals))


def pin_groupby_str_invariants(orc):
    rng = _rng(11)
    words, offsets, data = _strings(rng, 20_000, alphabet=4, maxlen=6)
    v = rng.integers(0, 10**6, size=20_000).astype(np.int64)
    rows, _, (s, c) = orc.groupby_str(offsets, data, [v], [("sum", 0), ("count", None)])
    assert int(c.sum()) == 20_000 and int(s.sum()) == int(v.sum()), "sum COUNT, sum SUM"
    assert len(rows) == len(set(words)), "one group per distinct string"
    firsts = {}
    for i, w in enumerate(words):
        firsts.setdefault(w, i)
    assert sorted(rows.tolist()) == sorted(firsts.values()), "each group's first row"
    keys = [words[r].encode() for r in rows]
    assert keys == sorted(keys), "groups in byte order"


ALL_PINS = [
    pin_filter_brute_force, pin_filter_closed_forms, pin_join_brute_force, pin_join_closed_forms,
    pin_join_invariants, pin_groupby_brute_force, pin_groupby_closed_forms, pin_groupby_arithmetic,
    pin_pipeline_brute_force, pin_pipeline_invariants, pin_semi_join_brute_force,
    pin_semi_join_closed_forms, pin_gather, pin_topn_selection, pin_groupby_str_brute_force,
    pin_groupby_str_invariants,
]
