"""Python binding of librel.so (include/rel.h): argument marshalling only.

Torch supplies device memory and the current stream; every step of the
relational path runs in the library's HIP kernels. The library must have
been built (``__graft_entry__.build()``); importing this module on a machine
without it, or calling an operator without a GPU, raises an error rather than
computing anything on the CPU.

Plans use plain Python values:
    preds : [(col, op, lo[, hi])]         op in lt le gt ge eq ne range
    aggs  : [(op, col)]                   op in sum count min max avg
    dims  : [dict(fk=fact col, key=tensor, payload=tensor or None)]
    keys  : [("fact", col) | ("dim", d)]
"""

from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librel.so")

REL_OK, REL_EINVAL, REL_ENOMEM, REL_ECAPACITY, REL_EDEVICE, REL_EUNSUPPORTED = range(6)
REL_F64 = 4
DTYPES = {torch.int8: 1, torch.int32: 2, torch.int64: 3}
TORCH_DTYPE = {1: torch.int8, 2: torch.int32, 3: torch.int64}
CMP = {"lt": 0, "le": 1, "gt": 2, "ge": 3, "eq": 4, "ne": 5, "range": 6}
AGG = {"sum": 0, "count": 1, "min": 2, "max": 3, "avg": 4}
MAX_TERMS, MAX_DIMS, MAX_KEYS, MAX_AGGS, MAX_FACT_COLS = 4, 2, 2, 8, 8


class RelError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"rel status {status}: {message}")
        self.status = status


class Column(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("idx", ctypes.c_void_p), ("len", ctypes.c_int64),
                ("type", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Pred(ctypes.Structure):
    _fields_ = [("col", ctypes.c_int32), ("op", ctypes.c_int32), ("lo", ctypes.c_int64),
                ("hi", ctypes.c_int64)]


class Agg(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("col", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("load_factor", ctypes.c_float), ("block", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("lds_slots", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("dim_lds_bytes", ctypes.c_int32),
                ("chunk_tiles", ctypes.c_int32), ("replicas", ctypes.c_int32),
                ("fanout", ctypes.c_int32)]


class Dim(ctypes.Structure):
    _fields_ = [("fact_col", ctypes.c_int32), ("has_payload", ctypes.c_int32), ("key", Column),
                ("payload", Column)]


class KeyRef(ctypes.Structure):
    _fields_ = [("src", ctypes.c_int32), ("col", ctypes.c_int32)]


class PipelineDesc(ctypes.Structure):
    _fields_ = [("fact", ctypes.POINTER(Column)), ("n_fact", ctypes.c_int32),
                ("preds", ctypes.POINTER(Pred)), ("n_preds", ctypes.c_int32),
                ("dims", ctypes.POINTER(Dim)), ("n_dims", ctypes.c_int32),
                ("keys", ctypes.POINTER(KeyRef)), ("n_keys", ctypes.c_int32),
                ("aggs", ctypes.POINTER(Agg)), ("n_aggs", ctypes.c_int32),
                ("max_groups", ctypes.c_int64), ("tuning", ctypes.POINTER(Tuning))]


class Strings(ctypes.Structure):
    _fields_ = [("offsets", ctypes.c_void_p), ("bytes", ctypes.c_void_p), ("codes", ctypes.c_void_p),
                ("len", ctypes.c_int64), ("n_strings", ctypes.c_int64)]


class Outputs(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p * MAX_KEYS), ("aggs", ctypes.c_void_p * MAX_AGGS),
                ("cap", ctypes.c_int64), ("d_groups", ctypes.c_void_p)]


# Every symbol include/rel.h declares: (name, restype, argtypes).
_P, _I, _L, _S = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
SIGNATURES = {
    "rel_status_str": (ctypes.c_char_p, [_I]),
    "rel_last_error": (ctypes.c_char_p, []),
    "rel_version": (_I, []),
    "rel_filter_ws": (_S, [_L]),
    "rel_filter": (_I, [_P, _I, _P, _I, _P, _L, _P, _P, _S, _P]),
    "rel_hash_join_ws": (_S, [ctypes.c_int32, _L, _P]),
    "rel_hash_join": (_I, [_P, _P, _P, _P, _L, _P, _P, _P, _S, _P]),
    "rel_groupby_ws": (_S, [_I, _P, _I, _P, _L, _L, _P]),
    "rel_groupby_agg": (_I, [_P, _I, _P, _I, _P, _I, _P, _P, _L, _P, _L, _P, _P, _S, _P]),
    "rel_pipeline_ws": (_S, [_P]),
    "rel_pipeline": (_I, [_P, _P, _P, _S, _P]),
    "rel_pipeline_batch_ws": (_S, [_P, _I]),
    "rel_pipeline_batch": (_I, [_P, _I, _P, _P, _S, _P]),
    "rel_pipeline_batch_graph": (_I, [_P, _I, _P, _P, _S, _P]),
    "rel_graph_launch": (_I, [_P, _P]),
    "rel_graph_destroy": (None, [_P]),
    "rel_server_create": (_I, [_P, _P]),
    "rel_server_submit": (_I, [_P, _P, _P, _P, _P]),
    "rel_server_poll": (_I, [_P, _P, _I]),
    "rel_server_drain": (_I, [_P, _L]),
    "rel_server_stats": (_I, [_P, _P, _P, _P, _P]),
    "rel_server_now_ns": (_L, []),
    "rel_server_destroy": (None, [_P]),
    "rel_kernel_name": (ctypes.c_char_p, [_I]),
    "rel_profile_enable": (None, [_I]),
    "rel_profile_read": (_I, [_P, _P]),
    "rel_stream_read": (_I, [_P, _L, _P, _P]),
    "rel_filter_noalloc": (_I, [_P, _I, _P, _I, _P, _L, _P, _P]),
    "rel_filter_sync": (_I, [_P, _I, _P, _I, _P, _L, _P, _P, _S, _P, _P]),
    "rel_hash_join_sync": (_I, [_P, _P, _P, _P, _L, _P, _P, _P, _S, _P, _P]),
    "rel_groupby_agg_sync": (_I, [_P, _I, _P, _I, _P, _I, _P, _P, _L, _P, _L, _P, _P, _S, _P,
                                  _P]),
    "rel_pipeline_sync": (_I, [_P, _P, _P, _S, _P, _P]),
    "rel_autotune": (_I, [_P, _I, ctypes.c_char_p]),
    "rel_autotune_lookup": (_I, [ctypes.c_char_p, _P, _P, _P]),
    "rel_bloom_bytes": (_S, [_L, ctypes.c_int32]),
    "rel_bloom_build": (_I, [_P, _P, _S, _P]),
    "rel_bloom_filter": (_I, [_P, _P, _S, _P, _L, _P, _P, _S, _P]),
    "rel_gather": (_I, [_P, _I, _P, _L, _P, _P]),
    "rel_topn_ws": (_S, [_L, _L]),
    "rel_topn": (_I, [_P, ctypes.c_int32, ctypes.c_int32, _P, _I, _L, _L, _P, _P, _P, _S, _P]),
    "rel_groupby_str_ws": (_S, [_L, _L, _I, _P]),
    "rel_groupby_str": (_I, [_P, _P, _P, _I, _P, _I, _P, _P, _P, _L, _P, _L, _P, _S, _P]),
    "rel_pipeline_stream_ws": (_S, [_P, _L]),
    "rel_pipeline_stream": (_I, [_P, _L, _P, _P, _S, _P]),
}

_lib = None


def lib():
    """The loaded librel.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def _check(status: int):
    if status != REL_OK:
        raise RelError(status, lib().rel_last_error().decode())


def _require_gpu(*tensors):
    if not torch.cuda.is_available():
        raise RuntimeError("the relational kernels need a ROCm GPU; none is visible")
    for t in tensors:
        if t is not None and not t.is_cuda:
            raise ValueError("inputs must be device tensors")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _addr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def column(t: torch.Tensor, idx: torch.Tensor | None = None) -> Column:
    if t.dtype not in DTYPES:
        raise TypeError(f"columns must be int8/int32/int64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("columns must be contiguous")
    if idx is not None:
        if idx.dtype != torch.int32 or not idx.is_contiguous():
            raise TypeError("row ids must be a contiguous int32 tensor holding uint32 values")
        return Column(t.data_ptr() if t.numel() else None, idx.data_ptr() if idx.numel() else None,
                      idx.numel(), DTYPES[t.dtype], 0)
    return Column(t.data_ptr() if t.numel() else None, None, t.numel(), DTYPES[t.dtype], 0)


TUNE_NO_DIRECT = 1
TUNE_BLOOM = 2


def tuning(load_factor=0.0, block=0, grid=0, lds_slots=0, dim_lds_bytes=0,
           chunk_tiles=0, replicas=0, flags=0, fanout=0) -> Tuning:
    return Tuning(load_factor, block, grid, lds_slots, flags, dim_lds_bytes, chunk_tiles, replicas,
                  fanout)


def _tuning_ptr(t):
    return ctypes.byref(t) if t is not None else None


def _arr(ctype, items):
    return (ctype * max(1, len(items)))(*items)


def _preds(preds):
    return _arr(Pred, [Pred(int(p[0]), CMP[p[1]], int(p[2]),
                            int(p[3]) if len(p) > 3 and p[3] is not None else 0) for p in preds])


def _aggs(aggs):
    return _arr(Agg, [Agg(AGG[op], int(col) if col is not None else 0) for op, col in aggs])


def workspace(nbytes: int, device=None) -> torch.Tensor:
    """A 256-byte aligned device buffer (torch's caching allocator aligns to 512)."""
    return torch.empty(max(256, int(nbytes)), dtype=torch.uint8, device=device or "cuda")


def _count(t: torch.Tensor) -> int:
    return int(t.item())


# -------------------------------------------------------------------- filter

def filter_ws(n: int) -> int:
    return int(lib().rel_filter_ws(n))


def filter_async(cols, preds, out, d_count, ws, idx=None):
    """Enqueues rel_filter; no allocation, no synchronisation."""
    ccols = _arr(Column, [column(c, idx) for c in cols])
    cp = _preds(preds)
    _check(lib().rel_filter(ccols, len(cols), cp, len(preds), _addr(out), out.numel(),
                            _addr(d_count), _addr(ws), ws.numel(), _stream()))


def filter_noalloc_async(cols, preds, out, d_count, idx=None):
    """Enqueues rel_filter_noalloc (tile states in the library's static
    device scratch; no workspace)."""
    ccols = _arr(Column, [column(c, idx) for c in cols])
    cp = _preds(preds)
    _check(lib().rel_filter_noalloc(ccols, len(cols), cp, len(preds), _addr(out), out.numel(),
                                    _addr(d_count), _stream()))


def filter(cols, preds, idx=None) -> torch.Tensor:
    """Row ids (int32 tensor holding uint32 values) of the passing elements,
    ascending."""
    _require_gpu(*cols)
    n = idx.numel() if idx is not None else cols[0].numel()
    out = torch.empty(max(1, n), dtype=torch.int32, device=cols[0].device)
    d_count = torch.zeros(1, dtype=torch.int64, device=cols[0].device)
    ws = workspace(filter_ws(n), cols[0].device)
    ccols = _arr(Column, [column(c, idx) for c in cols])
    cnt = ctypes.c_int64()
    _check(lib().rel_filter_sync(ccols, len(cols), _preds(preds), len(preds), _addr(out),
                                 out.numel(), _addr(d_count), _addr(ws), ws.numel(), _stream(),
                                 ctypes.byref(cnt)))
    return out[:cnt.value]


# ------------------------------------------------------------- Bloom filter

def bloom_bytes(n_keys: int, bits_per_key: int = 0) -> int:
    return int(lib().rel_bloom_bytes(n_keys, bits_per_key))


def bloom_build(keys: torch.Tensor, bits_per_key: int = 0, idx=None) -> torch.Tensor:
    """Blocked Bloom filter (uint8 device tensor) over the keys."""
    _require_gpu(keys)
    n = idx.numel() if idx is not None else keys.numel()
    f = workspace(bloom_bytes(n, bits_per_key), keys.device)
    c = column(keys, idx)
    _check(lib().rel_bloom_build(ctypes.byref(c), _addr(f), f.numel(), _stream()))
    return f


def bloom_filter_async(keys, filt, out, d_count, ws, idx=None):
    c = column(keys, idx)
    _check(lib().rel_bloom_filter(ctypes.byref(c), _addr(filt), filt.numel(), _addr(out),
                                  out.numel(), _addr(d_count), _addr(ws), ws.numel(), _stream()))


def bloom_filter(keys: torch.Tensor, filt: torch.Tensor, idx=None) -> torch.Tensor:
    """Row ids (ascending) of the keys that may be in the filter."""
    _require_gpu(keys)
    n = idx.numel() if idx is not None else keys.numel()
    out = torch.empty(max(1, n), dtype=torch.int32, device=keys.device)
    d_count = torch.zeros(1, dtype=torch.int64, device=keys.device)
    ws = workspace(filter_ws(n), keys.device)
    bloom_filter_async(keys, filt, out, d_count, ws, idx)
    return out[:_count(d_count)]


# ------------------------------------------------------ late materialisation

def gather_async(cols, ids, out, n=None):
    """out[c][i] = cols[c][ids[i]] for i < n (default: all of ids)."""
    n = ids.numel() if n is None else n
    cc = _arr(Column, [column(c) for c in cols])
    oo = _arr(ctypes.c_void_p, [o.data_ptr() for o in out])
    _check(lib().rel_gather(cc, len(cols), _addr(ids), n, oo, _stream()))


def gather(cols, ids):
    """Columns materialised at the row ids (each in its own dtype)."""
    _require_gpu(*cols)
    out = [torch.empty(ids.numel(), dtype=c.dtype, device=c.device) for c in cols]
    if ids.numel():
        gather_async(cols, ids, out)
    return out


def topn_ws(n: int, limit: int) -> int:
    return int(lib().rel_topn_ws(n, limit))


def topn_async(order, keys, limit, out, d_count, ws, desc=True):
    n = order.numel()
    ck = _arr(Column, [column(k) for k in keys])
    ot = REL_F64 if order.dtype == torch.float64 else DTYPES[order.dtype]
    _check(lib().rel_topn(_addr(order), ot, 1 if desc else 0, ck, len(keys), n, limit, _addr(out),
                          _addr(d_count), _addr(ws), ws.numel(), _stream()))


def topn(order: torch.Tensor, keys, limit: int, desc: bool = True) -> torch.Tensor:
    """Row positions of the first `limit` rows ordered by `order` (int64 or
    float64; descending by default), ties by the key tuple, then position."""
    _require_gpu(order, *keys)
    out = torch.empty(max(1, limit), dtype=torch.int32, device=order.device)
    d_count = torch.zeros(1, dtype=torch.int64, device=order.device)
    ws = workspace(topn_ws(order.numel(), limit), order.device)
    topn_async(order, keys, limit, out, d_count, ws, desc)
    return out[:_count(d_count)]


# ----------------------------------------------------------------- hash join

def hash_join_ws(key_type: torch.dtype, n_build: int, t: Tuning | None = None) -> int:
    return int(lib().rel_hash_join_ws(DTYPES[key_type], n_build, _tuning_ptr(t)))


def hash_join_async(build, probe, out_build, out_probe, d_count, ws, build_idx=None,
                    probe_idx=None, t: Tuning | None = None):
    cb, cp = column(build, build_idx), column(probe, probe_idx)
    _check(lib().rel_hash_join(ctypes.byref(cb), ctypes.byref(cp), _addr(out_build),
                               _addr(out_probe), out_build.numel(), _addr(d_count),
                               _tuning_ptr(t), _addr(ws), ws.numel(), _stream()))


def hash_join(build, probe, build_idx=None, probe_idx=None, out_cap=None,
              t: Tuning | None = None):
    """(build row ids, probe row ids) of every matching pair, unordered."""
    _require_gpu(build, probe)
    dev = probe.device
    n_build = build_idx.numel() if build_idx is not None else build.numel()
    n_probe = probe_idx.numel() if probe_idx is not None else probe.numel()
    ws = workspace(hash_join_ws(build.dtype, n_build, t), dev)
    d_count = torch.zeros(1, dtype=torch.int64, device=dev)
    cap = max(1, n_probe if out_cap is None else out_cap)
    cb, cp = column(build, build_idx), column(probe, probe_idx)
    total = ctypes.c_int64()
    while True:
        ob = torch.empty(cap, dtype=torch.int32, device=dev)
        op = torch.empty(cap, dtype=torch.int32, device=dev)
        st = lib().rel_hash_join_sync(ctypes.byref(cb), ctypes.byref(cp), _addr(ob), _addr(op),
                                      cap, _addr(d_count), _tuning_ptr(t), _addr(ws), ws.numel(),
                                      _stream(), ctypes.byref(total))
        if st == REL_ECAPACITY:
            cap = total.value  # more pairs than the output holds: grow it and join again
            continue
        _check(st)
        return ob[:total.value], op[:total.value]


# ------------------------------------------------------------------ group-by

def _out_tensors(key_dtypes, aggs, cap, dev):
    out_keys = [torch.empty(cap, dtype=dt, device=dev) for dt in key_dtypes]
    out_aggs = [torch.empty(cap, dtype=torch.float64 if op == "avg" else torch.int64, device=dev)
                for op, _ in aggs]
    return out_keys, out_aggs


def groupby_ws(key_dtypes, aggs, n_rows: int, max_groups: int, t: Tuning | None = None) -> int:
    kt = _arr(ctypes.c_int32, [DTYPES[d] for d in key_dtypes])
    return int(lib().rel_groupby_ws(len(key_dtypes), kt, len(aggs), _aggs(aggs), n_rows,
                                    max_groups, _tuning_ptr(t)))


def groupby_agg_async(keys, vals, aggs, out_keys, out_aggs, d_groups, max_groups, ws,
                      key_idx=None, val_idx=None, t: Tuning | None = None):
    ck = _arr(Column, [column(k, key_idx) for k in keys])
    cv = _arr(Column, [column(v, val_idx) for v in vals])
    ok = _arr(ctypes.c_void_p, [o.data_ptr() for o in out_keys])
    oa = _arr(ctypes.c_void_p, [o.data_ptr() for o in out_aggs])
    cap = out_aggs[0].numel() if out_aggs else 0
    _check(lib().rel_groupby_agg(ck, len(keys), cv, len(vals), _aggs(aggs), len(aggs), ok, oa, cap,
                                 _addr(d_groups), max_groups, _tuning_ptr(t), _addr(ws),
                                 ws.numel(), _stream()))


def groupby_agg(keys, vals, aggs, max_groups: int | None = None, key_idx=None, val_idx=None,
                t: Tuning | None = None):
    """(key columns, aggregate columns) of every group, unordered."""
    _require_gpu(*keys, *vals)
    dev = (keys or vals)[0].device
    n = key_idx.numel() if key_idx is not None else (keys or vals)[0].numel()
    max_groups = max(1, n) if max_groups is None else max_groups
    key_dtypes = [k.dtype for k in keys]
    ws = workspace(groupby_ws(key_dtypes, aggs, n, max_groups, t), dev)
    d_groups = torch.zeros(1, dtype=torch.int64, device=dev)
    cap = max(1, min(max_groups, max(1, n)))
    ck = _arr(Column, [column(k, key_idx) for k in keys])
    cv = _arr(Column, [column(v, val_idx) for v in vals])
    ng = ctypes.c_int64()
    while True:
        out_keys, out_aggs = _out_tensors(key_dtypes, aggs, cap, dev)
        ok = _arr(ctypes.c_void_p, [o.data_ptr() for o in out_keys])
        oa = _arr(ctypes.c_void_p, [o.data_ptr() for o in out_aggs])
        st = lib().rel_groupby_agg_sync(ck, len(keys), cv, len(vals), _aggs(aggs), len(aggs), ok,
                                        oa, cap, _addr(d_groups), max_groups, _tuning_ptr(t),
                                        _addr(ws), ws.numel(), _stream(), ctypes.byref(ng))
        if st == REL_ECAPACITY and ng.value < 0:
            raise RelError(REL_ECAPACITY, f"more than max_groups={max_groups} groups")
        if st == REL_ECAPACITY:
            cap = ng.value
            continue
        _check(st)
        return [k[:ng.value] for k in out_keys], [a[:ng.value] for a in out_aggs]


# ------------------------------------------------------- string group-by

def strings(offsets: torch.Tensor, data: torch.Tensor, codes: torch.Tensor | None = None) -> Strings:
    """A string column (Arrow layout: int64 offsets, uint8 bytes), optionally
    dictionary-encoded by int32 codes."""
    if offsets.dtype != torch.int64 or data.dtype != torch.uint8:
        raise TypeError("strings need int64 offsets and uint8 bytes")
    ns = offsets.numel() - 1
    n = codes.numel() if codes is not None else ns
    return Strings(_addr(offsets), data.data_ptr() if data.numel() else _addr(offsets),
                   _addr(codes) if codes is not None else None, n, ns)


def groupby_str_ws(aggs, max_groups: int, n_dict: int = 0) -> int:
    """Workspace bytes; n_dict = the dictionary's string count for a
    dictionary-encoded column, 0 otherwise."""
    return int(lib().rel_groupby_str_ws(max_groups, n_dict, len(aggs), _aggs(aggs)))


def groupby_str(offsets, data, vals, aggs, ikey=None, codes=None, max_groups: int | None = None):
    """(first row ids, int keys or None, aggregate columns) per distinct
    (string, int key); order unspecified."""
    _require_gpu(offsets, data, *vals)
    dev = offsets.device
    st = strings(offsets, data, codes)
    n = st.len
    max_groups = max(1, n) if max_groups is None else max_groups
    ws = workspace(groupby_str_ws(aggs, max_groups, st.n_strings if codes is not None else 0), dev)
    cv = _arr(Column, [column(v) for v in vals])
    ck = column(ikey) if ikey is not None else None
    d_groups = torch.zeros(1, dtype=torch.int64, device=dev)
    cap = max(1, min(max_groups, max(1, n)))
    while True:
        rows = torch.empty(cap, dtype=torch.int32, device=dev)
        iks = torch.empty(cap, dtype=ikey.dtype, device=dev) if ikey is not None else None
        out_aggs = [torch.empty(cap, dtype=torch.float64 if op == "avg" else torch.int64, device=dev)
                    for op, _ in aggs]
        oa = _arr(ctypes.c_void_p, [o.data_ptr() for o in out_aggs])
        _check(lib().rel_groupby_str(ctypes.byref(st), ctypes.byref(ck) if ck is not None else None,
                                     cv, len(vals), _aggs(aggs), len(aggs), _addr(rows),
                                     _addr(iks) if iks is not None else None, oa, cap,
                                     _addr(d_groups), max_groups, _addr(ws), ws.numel(), _stream()))
        ng = _count(d_groups)
        if ng < 0:
            raise RelError(REL_ECAPACITY, f"more than max_groups={max_groups} groups")
        if ng <= cap:
            return rows[:ng], (iks[:ng] if iks is not None else None), [a[:ng] for a in out_aggs]
        cap = ng


# ------------------------------------------------------------------ pipeline

class Plan:
    """A fused plan bound to its inputs and output buffers (no workspace)."""

    def __init__(self, fact, preds, dims, keys, aggs, max_groups: int, t: Tuning | None = None,
                 out_cap: int | None = None, host_fact: bool = False):
        if host_fact:
            # fact columns in (pinned) host memory, streamed by rel_pipeline_stream
            if not torch.cuda.is_available():
                raise RuntimeError("the relational kernels need a ROCm GPU; none is visible")
            dev = dims[0]["key"].device if dims else torch.device("cuda", torch.cuda.current_device())
        else:
            _require_gpu(*fact)
            dev = fact[0].device
        self.device = dev
        self._keep = [fact, dims]
        self.aggs = aggs
        self._fact = _arr(Column, [column(c) for c in fact])
        self._preds = _preds(preds)
        cdims = []
        for d in dims:
            pay = d.get("payload")
            cdims.append(Dim(int(d["fk"]), 1 if pay is not None else 0, column(d["key"]),
                             column(pay) if pay is not None else Column()))
        self._dims = _arr(Dim, cdims)
        self._keys = _arr(KeyRef, [KeyRef(0 if src == "fact" else 1, int(c)) for src, c in keys])
        self._aggs = _aggs(aggs)
        self._tuning = t
        self.desc = PipelineDesc(
            ctypes.cast(self._fact, ctypes.POINTER(Column)), len(fact),
            ctypes.cast(self._preds, ctypes.POINTER(Pred)), len(preds),
            ctypes.cast(self._dims, ctypes.POINTER(Dim)), len(dims),
            ctypes.cast(self._keys, ctypes.POINTER(KeyRef)), len(keys),
            ctypes.cast(self._aggs, ctypes.POINTER(Agg)), len(aggs), int(max_groups),
            ctypes.pointer(t) if t is not None else None)
        key_dtypes = [fact[c].dtype if src == "fact" else dims[c]["payload"].dtype
                      for src, c in keys]
        self.key_dtypes = key_dtypes
        self.cap = max(1, int(max_groups) if out_cap is None else out_cap)
        self.out_keys, self.out_aggs = _out_tensors(key_dtypes, aggs, self.cap, dev)
        self.d_groups = torch.zeros(1, dtype=torch.int64, device=dev)
        self.outputs = Outputs()
        for i, k in enumerate(self.out_keys):
            self.outputs.keys[i] = k.data_ptr()
        for i, a in enumerate(self.out_aggs):
            self.outputs.aggs[i] = a.data_ptr()
        self.outputs.cap = self.cap
        self.outputs.d_groups = self.d_groups.data_ptr()

    def result(self):
        """Synchronises on the group count and returns (keys, aggs)."""
        ng = _count(self.d_groups)
        if ng < 0:
            raise RelError(REL_ECAPACITY, "more groups than max_groups")
        if ng > self.cap:
            raise RelError(REL_ECAPACITY, f"{ng} groups exceed the output capacity {self.cap}")
        return [k[:ng] for k in self.out_keys], [a[:ng] for a in self.out_aggs]


class PreparedPipeline(Plan):
    """A fused plan with its own workspace. ``launch()`` only enqueues
    kernels (no allocation, no synchronisation)."""

    def __init__(self, *args, **kwargs):
        super().__init__(*args, **kwargs)
        nbytes = lib().rel_pipeline_ws(ctypes.byref(self.desc))
        if nbytes == 0:
            # the same validation, run again, names the problem
            _check(lib().rel_pipeline(ctypes.byref(self.desc), None, None, 0, None))
        self.ws = workspace(nbytes, self.device)

    def launch(self):
        _check(lib().rel_pipeline(ctypes.byref(self.desc), ctypes.byref(self.outputs),
                                  _addr(self.ws), self.ws.numel(), _stream()))

    def run(self):
        """rel_pipeline_sync: runs the plan, waits, returns (keys, aggs)."""
        ng = ctypes.c_int64()
        _check(lib().rel_pipeline_sync(ctypes.byref(self.desc), ctypes.byref(self.outputs),
                                       _addr(self.ws), self.ws.numel(), _stream(),
                                       ctypes.byref(ng)))
        return [k[:ng.value] for k in self.out_keys], [a[:ng.value] for a in self.out_aggs]


class PreparedBatch:
    """Plans of one shape run together by rel_pipeline_batch, sharing one
    workspace; each plan keeps its own outputs (``Plan.result()``).
    ``launch()`` enqueues the batch; ``capture()`` records it once as a graph
    that ``launch_graph()`` replays."""

    def __init__(self, plans: list):
        if not plans:
            raise ValueError("a batch needs at least one plan")
        self.plans = plans
        n = len(plans)
        self.n = n
        self.descs = (PipelineDesc * n)(*[p.desc for p in plans])
        self.outs = (Outputs * n)(*[p.outputs for p in plans])
        nbytes = lib().rel_pipeline_batch_ws(self.descs, n)
        if nbytes == 0:
            _check(lib().rel_pipeline_batch(self.descs, n, None, None, 0, None))
        self.ws = workspace(nbytes, plans[0].device)
        self._graph = None

    def launch(self):
        _check(lib().rel_pipeline_batch(self.descs, self.n, self.outs, _addr(self.ws),
                                        self.ws.numel(), _stream()))

    def capture(self):
        """Captures the batch as a graph (nothing runs)."""
        self.release()
        g = ctypes.c_void_p()
        _check(lib().rel_pipeline_batch_graph(self.descs, self.n, self.outs, _addr(self.ws),
                                              self.ws.numel(), ctypes.byref(g)))
        self._graph = g

    def launch_graph(self):
        if self._graph is None:
            raise RuntimeError("capture() the batch first")
        _check(lib().rel_graph_launch(self._graph, _stream()))

    def release(self):
        """Destroys the captured graph (after synchronising the device)."""
        if self._graph is not None:
            torch.cuda.synchronize(self.plans[0].device)
            lib().rel_graph_destroy(self._graph)
            self._graph = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def results(self):
        return [p.result() for p in self.plans]


class StreamedPipeline(Plan):
    """A fused plan over fact columns in host memory (pinned CPU tensors),
    streamed through the device in chunks by rel_pipeline_stream."""

    def __init__(self, fact, preds, dims, keys, aggs, max_groups: int, chunk_rows: int,
                 t: Tuning | None = None):
        for c in fact:
            if c.is_cuda:
                raise ValueError("streamed fact columns live in host memory")
        super().__init__(fact, preds, dims, keys, aggs, max_groups, t, host_fact=True)
        self.chunk_rows = chunk_rows
        nbytes = lib().rel_pipeline_stream_ws(ctypes.byref(self.desc), chunk_rows)
        if nbytes == 0:
            _check(lib().rel_pipeline_stream(ctypes.byref(self.desc), chunk_rows, None, None, 0,
                                             None))
        self.ws = workspace(nbytes, self.device)

    def launch(self):
        _check(lib().rel_pipeline_stream(ctypes.byref(self.desc), self.chunk_rows,
                                         ctypes.byref(self.outputs), _addr(self.ws),
                                         self.ws.numel(), _stream()))


def pipeline(fact, preds, dims, keys, aggs, max_groups: int, t: Tuning | None = None):
    """Runs the fused plan and returns (key columns, aggregate columns)."""
    return PreparedPipeline(fact, preds, dims, keys, aggs, max_groups, t).run()


# ---------------------------------------------------------------- stream read

def stream_read_async(t: torch.Tensor, d_xor: torch.Tensor, nbytes: int | None = None):
    """Reads the first nbytes bytes of t's storage once (default: all of t);
    d_xor (one int64 on the device) receives the XOR of its 64-bit words."""
    _require_gpu(t, d_xor)
    n = t.numel() * t.element_size() if nbytes is None else nbytes
    _check(lib().rel_stream_read(_addr(t), n, _addr(d_xor), _stream()))


def stream_read(t: torch.Tensor) -> int:
    """XOR of the 64-bit words of t's bytes (zero-padded), read on the GPU."""
    d = torch.zeros(1, dtype=torch.int64, device=t.device)
    stream_read_async(t, d)
    return int(d.item()) & ((1 << 64) - 1)


# ------------------------------------------------------------------ profiling

KERNEL_CLASSES = 12


def profile_enable(on: bool = True):
    """Brackets every kernel launched afterwards with HIP events."""
    lib().rel_profile_enable(1 if on else 0)


def profile_read() -> dict:
    """{kernel class: (total ms, launches)} since the last read (synchronises)."""
    ms = (ctypes.c_double * KERNEL_CLASSES)()
    n = (ctypes.c_int64 * KERNEL_CLASSES)()
    _check(lib().rel_profile_read(ms, n))
    return {lib().rel_kernel_name(k).decode(): (ms[k], n[k]) for k in range(KERNEL_CLASSES)}
