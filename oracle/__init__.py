"""Plain single-threaded CPU oracle for the relational hot path (filter ->
hash join -> hash group-by) of arXiv 2508.04701, Section 3.2.2.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``, never by the product package.
It wraps ``oracle.cpp`` (std::unordered_map join and group-by, one row at a
time) and shares no code with the HIP path.

Arrays are numpy; element types are int8 / int32 / int64. Plans use the same
plain-Python description as the tests:

    terms : [(col, op, lo, hi)]   op in lt le gt ge eq ne range
    aggs  : [(op, col)]           op in sum count min max avg
    keys  : [("fact", col)] or [("dim", d)]   (pipeline group keys)

Results come back in canonical order: filter in scan order, join pairs sorted
by (probe row, build row), groups sorted by key tuple.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_TYPES = {np.dtype(np.int8): 1, np.dtype(np.int32): 2, np.dtype(np.int64): 3}
CMP_OPS = {"lt": 0, "le": 1, "gt": 2, "ge": 3, "eq": 4, "ne": 5, "range": 6}
AGG_OPS = {"sum": 0, "count": 1, "min": 2, "max": 3, "avg": 4}



def build(src: str = _SRC, out: str = _LIB_PATH) -> str:
    """Compiles oracle.cpp (or a given variant of it) with g++; no GPU involved."""
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", out + ".tmp", src]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _open(path: str):
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I = ctypes.c_int
    L = ctypes.c_int64
    lib.oracle_filter.restype = L
    lib.oracle_filter.argtypes = [I, P, P, L, P, L, I, P, P, P, P, P]
    lib.oracle_hash_join.restype = L
    lib.oracle_hash_join.argtypes = [P, P, I, L, L, P, P, L]
    lib.oracle_groupby.restype = L
    lib.oracle_groupby.argtypes = [I, P, P, I, P, P, I, P, P, L, P, P, L]
    lib.oracle_pipeline.restype = L
    lib.oracle_pipeline.argtypes = [I, P, P, L, I, P, P, P, P, I, P, P, P, P, P, P,
                                    I, P, P, I, P, P, P, P, L]
    lib.oracle_semi_join.restype = L
    lib.oracle_semi_join.argtypes = [P, P, I, L, L, P]
    lib.oracle_gather.restype = None
    lib.oracle_gather.argtypes = [P, I, P, L, P]
    lib.oracle_topn.restype = L
    lib.oracle_topn.argtypes = [L, P, I, I, I, P, L, P]
    lib.oracle_groupby_str.restype = L
    lib.oracle_groupby_str.argtypes = [L, P, P, P, I, I, P, P, I, P, P, P, P, P, L]
    return lib


def _col(a) -> np.ndarray:
    a = np.ascontiguousarray(a)
    if a.dtype not in _TYPES:
        raise TypeError(f"oracle columns must be int8/int32/int64, got {a.dtype}")
    return a


class _Arr:
    """Keeps numpy arrays alive while ctypes holds raw pointers into them."""

    def __init__(self):
        self.keep = []

    def ptr(self, a):
        if a is None:
            return None
        self.keep.append(a)
        return a.ctypes.data

    def ints(self, vals, dtype=np.int32):
        a = np.ascontiguousarray(np.asarray(list(vals), dtype=dtype))
        if a.size == 0:
            a = np.zeros(1, dtype=dtype)
        return self.ptr(a)

    def ptrs(self, arrays):
        p = (ctypes.c_void_p * max(1, len(arrays)))()
        for i, a in enumerate(arrays):
            p[i] = self.ptr(a) if a is not None else None
        self.keep.append(p)
        return ctypes.cast(p, ctypes.c_void_p).value


def _terms(k: _Arr, terms):
    terms = list(terms)
    cols = [t[0] for t in terms]
    ops = [CMP_OPS[t[1]] for t in terms]
    lo = [int(t[2]) for t in terms]
    hi = [int(t[3]) if len(t) > 3 and t[3] is not None else 0 for t in terms]
    return (len(terms), k.ints(cols), k.ints(ops), k.ints(lo, np.int64), k.ints(hi, np.int64))


class Oracle:
    """The oracle functions bound to one build of oracle.cpp."""

    def __init__(self, lib_path: str = _LIB_PATH):
        if lib_path == _LIB_PATH and not os.path.exists(lib_path):
            build()
        self.lib = _open(lib_path)

    def filter(self, cols, terms, sel=None) -> np.ndarray:
        """Row ids (uint32) of the rows satisfying every term, in scan order."""
        return _filter(self.lib, cols, terms, sel)

    def hash_join(self, build, probe):
        """All pairs (build row, probe row) with equal keys, sorted by (probe, build)."""
        return _hash_join(self.lib, build, probe)

    def groupby(self, keys, vals, aggs):
        """(key columns, aggregate columns) sorted by key tuple."""
        return _groupby(self.lib, keys, vals, aggs)

    def pipeline(self, fact, terms, dims, keys, aggs):
        """Fused filter -> inner join with up to two dims -> group-by."""
        return _pipeline(self.lib, fact, terms, dims, keys, aggs)

    def semi_join(self, build, probe):
        """Probe row ids (uint32, ascending) with at least one equal build key."""
        return _semi_join(self.lib, build, probe)

    def gather(self, col, idx):
        """col[idx[i]] widened to int64 (late materialisation)."""
        return _gather(self.lib, col, idx)

    def topn(self, order, keys, limit, desc=True):
        """Row positions of the first `limit` rows ordered by `order` (int64
        or float64; descending when desc), ties by the key tuple ascending."""
        return _topn(self.lib, order, keys, limit, desc)

    def groupby_str(self, offsets, data, vals, aggs, ikey=None):
        """Group-by on the string key (Arrow offsets/bytes) and optional int
        key: (first row ids, int keys, aggregate columns) by (string, int key)."""
        return _groupby_str(self.lib, offsets, data, vals, aggs, ikey)


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def filter(cols, terms, sel=None):
    return default().filter(cols, terms, sel)


def hash_join(build, probe):
    return default().hash_join(build, probe)


def groupby(keys, vals, aggs):
    return default().groupby(keys, vals, aggs)


def pipeline(fact, terms, dims, keys, aggs):
    return default().pipeline(fact, terms, dims, keys, aggs)


def semi_join(build, probe):
    return default().semi_join(build, probe)


def gather(col, idx):
    return default().gather(col, idx)


def topn(order, keys, limit, desc=True):
    return default().topn(order, keys, limit, desc)


def groupby_str(offsets, data, vals, aggs, ikey=None):
    return default().groupby_str(offsets, data, vals, aggs, ikey)


def _semi_join(lib, build, probe) -> np.ndarray:
    build, probe = _col(build), _col(probe)
    if build.dtype != probe.dtype:
        raise TypeError("build and probe key types differ")
    k = _Arr()
    out = np.empty(max(1, len(probe)), dtype=np.uint32)
    cnt = lib.oracle_semi_join(k.ptr(build), k.ptr(probe), _TYPES[build.dtype], len(build),
                               len(probe), k.ptr(out))
    return out[:cnt].copy()


def _gather(lib, col, idx) -> np.ndarray:
    col = _col(col)
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    k = _Arr()
    out = np.empty(max(1, len(idx)), dtype=np.int64)
    lib.oracle_gather(k.ptr(col), _TYPES[col.dtype], k.ptr(idx), len(idx), k.ptr(out))
    return out[:len(idx)].copy()


def _topn(lib, order, keys, limit, desc=True) -> np.ndarray:
    order = np.ascontiguousarray(order)
    if order.dtype not in (np.dtype(np.int64), np.dtype(np.float64)):
        raise TypeError("top-N orders by an int64 or float64 column")
    keys = [np.ascontiguousarray(c, dtype=np.int64) for c in keys]
    n = len(order)
    k = _Arr()
    out = np.empty(max(1, min(limit, n)), dtype=np.uint32)
    m = lib.oracle_topn(n, k.ptr(order), 1 if order.dtype == np.float64 else 0, 1 if desc else 0,
                        len(keys), k.ptrs(keys), int(limit), k.ptr(out))
    return out[:m].copy()


def _groupby_str(lib, offsets, data, vals, aggs, ikey=None):
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    data = np.ascontiguousarray(data, dtype=np.uint8)
    n = len(offsets) - 1
    vals = [_col(c) for c in vals]
    ik = None if ikey is None else _col(ikey)
    k = _Arr()
    vp, vt = k.ptrs(vals), k.ints([_TYPES[c.dtype] for c in vals])
    ao = k.ints([AGG_OPS[a[0]] for a in aggs])
    ac = k.ints([a[1] if a[1] is not None else 0 for a in aggs])
    cap = max(1, min(n, 1 << 16))
    while True:
        rows = np.zeros(cap, dtype=np.uint32)
        iks = np.zeros(cap, dtype=np.int64)
        out_aggs = np.zeros(max(1, len(aggs)) * cap, dtype=np.int64)
        ng = lib.oracle_groupby_str(n, k.ptr(offsets), k.ptr(data if len(data) else
                                                              np.zeros(1, np.uint8)),
                                    k.ptr(ik), 0 if ik is None else _TYPES[ik.dtype], len(vals),
                                    vp, vt, len(aggs), ao, ac, k.ptr(rows), k.ptr(iks),
                                    k.ptr(out_aggs), cap)
        if ng <= cap:
            break
        cap = ng
    return rows[:ng].copy(), iks[:ng].copy(), _agg_results(aggs, out_aggs, ng, cap)


def _filter(lib, cols, terms, sel=None) -> np.ndarray:
    cols = [_col(c) for c in cols]
    n = len(cols[0]) if cols else 0
    k = _Arr()
    sel_arr = None if sel is None else np.ascontiguousarray(sel, dtype=np.uint32)
    scan = n if sel_arr is None else len(sel_arr)
    out = np.empty(max(1, scan), dtype=np.uint32)
    nt, tc, to, tl, th = _terms(k, terms)
    cnt = lib.oracle_filter(len(cols), k.ptrs(cols), k.ints([_TYPES[c.dtype] for c in cols]), n,
                            k.ptr(sel_arr), 0 if sel_arr is None else len(sel_arr),
                            nt, tc, to, tl, th, k.ptr(out))
    return out[:cnt].copy()


def _hash_join(lib, build, probe):
    build, probe = _col(build), _col(probe)
    if build.dtype != probe.dtype:
        raise TypeError("build and probe key types differ")
    k = _Arr()
    kt = _TYPES[build.dtype]
    total = lib.oracle_hash_join(k.ptr(build), k.ptr(probe), kt, len(build), len(probe), None, None, 0)
    ob = np.empty(max(1, total), dtype=np.uint32)
    op = np.empty(max(1, total), dtype=np.uint32)
    lib.oracle_hash_join(k.ptr(build), k.ptr(probe), kt, len(build), len(probe),
                         k.ptr(ob), k.ptr(op), total)
    return ob[:total].copy(), op[:total].copy()


def _agg_results(aggs, raw, ng, cap):
    out = []
    for a, (op, _) in enumerate(aggs):
        col = raw[a * cap: a * cap + ng].copy()
        out.append(col.view(np.float64) if op == "avg" else col)
    return out


def _groupby_call(call, nkeys, aggs, size_hint):
    cap = max(1, size_hint)
    while True:
        out_keys = np.zeros(max(1, nkeys) * cap, dtype=np.int64)
        out_aggs = np.zeros(max(1, len(aggs)) * cap, dtype=np.int64)
        ng = call(out_keys, out_aggs, cap)
        if ng <= cap:
            break
        cap = ng
    keys = [out_keys[k * cap: k * cap + ng].copy() for k in range(nkeys)]
    return keys, _agg_results(aggs, out_aggs, ng, cap)


def _groupby(lib, keys, vals, aggs):
    """Groups rows by the key tuple; returns (key columns, aggregate columns).

    Key columns are int64; SUM/COUNT/MIN/MAX are int64 and AVG is float64."""
    keys = [_col(c) for c in keys]
    vals = [_col(c) for c in vals]
    n = len(keys[0]) if keys else (len(vals[0]) if vals else 0)
    k = _Arr()
    kp, kt = k.ptrs(keys), k.ints([_TYPES[c.dtype] for c in keys])
    vp, vt = k.ptrs(vals), k.ints([_TYPES[c.dtype] for c in vals])
    ao = k.ints([AGG_OPS[a[0]] for a in aggs])
    ac = k.ints([a[1] if a[1] is not None else 0 for a in aggs])

    def call(out_keys, out_aggs, cap):
        return lib.oracle_groupby(len(keys), kp, kt, len(vals), vp, vt, len(aggs), ao, ac, n,
                                  k.ptr(out_keys), k.ptr(out_aggs), cap)

    return _groupby_call(call, len(keys), aggs, min(n, 1 << 16) + 1)


def _pipeline(lib, fact, terms, dims, keys, aggs):
    """dims: [dict(fk=fact column index, key=dim key array, payload=array or None)]
    keys: [("fact", col)] or [("dim", d)]."""
    fact = [_col(c) for c in fact]
    n = len(fact[0]) if fact else 0
    k = _Arr()
    nt, tc, to, tl, th = _terms(k, terms)
    dkeys = [_col(d["key"]) for d in dims]
    dpay = [None if d.get("payload") is None else _col(d["payload"]) for d in dims]
    dpt = [0 if p is None else _TYPES[p.dtype] for p in dpay]
    key_src = [0 if src == "fact" else 1 + int(c) for src, c in keys]
    key_col = [int(c) if src == "fact" else 0 for src, c in keys]
    ao = k.ints([AGG_OPS[a[0]] for a in aggs])
    ac = k.ints([a[1] if a[1] is not None else 0 for a in aggs])
    fp, ft = k.ptrs(fact), k.ints([_TYPES[c.dtype] for c in fact])
    dfk = k.ints([d["fk"] for d in dims])
    dkp, dkt = k.ptrs(dkeys), k.ints([_TYPES[c.dtype] for c in dkeys])
    dn = k.ints([len(c) for c in dkeys], np.int64)
    dpp, dptp = k.ptrs(dpay), k.ints(dpt)
    ks, kc = k.ints(key_src), k.ints(key_col)

    def call(out_keys, out_aggs, cap):
        return lib.oracle_pipeline(len(fact), fp, ft, n, nt, tc, to, tl, th, len(dims), dfk, dkp,
                                   dkt, dn, dpp, dptp, len(keys), ks, kc, len(aggs), ao, ac,
                                   k.ptr(out_keys), k.ptr(out_aggs), cap)

    return _groupby_call(call, len(keys), aggs, 1 << 12)
