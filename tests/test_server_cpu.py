"""The serving scheduler (rel_server_*) on the CPU, driven by a test executor
that runs each batch with the oracle on the host and takes a fixed time per
batch. It checks what the scheduler promises: every query completes exactly
once with the result of its own plan; FIFO order within a shape; batches of
one shape within max_batch; in-flight queries within max_slots and lanes;
workspaces carved from the arena never overlap; oversized queries are
rejected while others go on; forced launch failures and executor failures
fail only their batch."""

import ctypes
import os
import threading
import time

import numpy as np
import pytest

import oracle
from paper_2508_04701_amd import rel, serve

ARENA_BASE = 1 << 40  # a fake device address: the test executor never dereferences it


class HostPlan:
    """A plan over host columns (the test executor reads them back by
    identity), with a description and outputs for the C-ABI."""

    def __init__(self, fact, terms, dims, keys, aggs, max_groups):
        self.spec = (fact, terms, dims, keys, aggs)
        self.arrays = [np.ascontiguousarray(c) for c in fact]
        cols = [rel.Column(a.ctypes.data if a.size else None, None, a.size,
                           rel.DTYPES[_torch_dtype(a)], 0) for a in self.arrays]
        self._fact = (rel.Column * len(cols))(*cols)
        self._preds = rel._preds(terms)
        self._dim_arrays = []
        cdims = []
        for d in dims:
            k = np.ascontiguousarray(d["key"])
            p = None if d.get("payload") is None else np.ascontiguousarray(d["payload"])
            self._dim_arrays += [k, p]
            cdims.append(rel.Dim(d["fk"], 1 if p is not None else 0,
                                 rel.Column(k.ctypes.data if k.size else None, None, k.size,
                                            rel.DTYPES[_torch_dtype(k)], 0),
                                 rel.Column(p.ctypes.data if p is not None and p.size else None,
                                            None, 0 if p is None else p.size,
                                            rel.DTYPES[_torch_dtype(p)] if p is not None else 0, 0)))
        self._dims = rel._arr(rel.Dim, cdims)
        self._keys = rel._arr(rel.KeyRef, [rel.KeyRef(0 if s == "fact" else 1, c) for s, c in keys])
        self._aggs = rel._aggs(aggs)
        self.desc = rel.PipelineDesc(
            ctypes.cast(self._fact, ctypes.POINTER(rel.Column)), len(cols),
            ctypes.cast(self._preds, ctypes.POINTER(rel.Pred)), len(terms),
            ctypes.cast(self._dims, ctypes.POINTER(rel.Dim)), len(dims),
            ctypes.cast(self._keys, ctypes.POINTER(rel.KeyRef)), len(keys),
            ctypes.cast(self._aggs, ctypes.POINTER(rel.Agg)), len(aggs), max_groups, None)
        self.count = np.zeros(1, np.int64)  # identifies the query in the executor
        self.outputs = rel.Outputs()
        self.outputs.cap = max_groups
        self.outputs.d_groups = self.count.ctypes.data
        self._out_bufs = [np.zeros(max_groups, np.int64) for _ in range(len(keys) + len(aggs))]
        for i in range(len(keys)):
            self.outputs.keys[i] = self._out_bufs[i].ctypes.data
        for i in range(len(aggs)):
            self.outputs.aggs[i] = self._out_bufs[len(keys) + i].ctypes.data
        self.result = None


def _torch_dtype(a):
    import torch
    return {np.dtype(np.int8): torch.int8, np.dtype(np.int32): torch.int32,
            np.dtype(np.int64): torch.int64}[a.dtype]


class OracleExecutor:
    """Runs a batch with the oracle when it is launched and reports it done
    `delay` seconds later; records what the scheduler asked for."""

    def __init__(self, plans, lanes, delay=0.003, fail_poll_at=None, fail_launch_at=None):
        self.by_count = {p.count.ctypes.data: p for p in plans}
        self.delay = delay
        self.lane_until = [None] * lanes
        self.lane_fail = [False] * lanes
        self.launches = []        # (time, lane, [plans], ws offset, ws bytes)
        self.active = {}          # lane -> (off, bytes, nqueries)
        self.max_active_queries = 0
        self.max_active_lanes = 0
        self.errors = []
        self.fail_poll_at = fail_poll_at
        self.fail_launch_at = fail_launch_at
        self.quiesced = []
        self.lock = threading.Lock()
        self.struct = serve.Executor(None, serve.BATCH_WS(self._ws), serve.LAUNCH(self._launch),
                                     serve.POLL(self._poll), serve.QUIESCE(self._quiesce))

    def _ws(self, user, d, n):
        return rel.lib().rel_pipeline_batch_ws(d, n)

    def _launch(self, user, lane, d, n, o, host, ws, ws_bytes):
        try:
            descs = ctypes.cast(d, ctypes.POINTER(rel.PipelineDesc))
            outs = ctypes.cast(o, ctypes.POINTER(rel.Outputs))
            batch = []
            for i in range(n):
                p = self.by_count[outs[i].d_groups]
                # the scheduler must pass each plan with its own outputs
                if descs[i].fact[0].data != p.desc.fact[0].data or \
                        descs[i].n_aggs != p.desc.n_aggs:
                    self.errors.append(f"plan/output mismatch in launch {len(self.launches)}")
                p.result = oracle.pipeline(*p.spec)
                batch.append(p)
            off = ws - ARENA_BASE
            with self.lock:
                if self.lane_until[lane] is not None:
                    self.errors.append(f"lane {lane} launched while busy")
                for other, (o2, b2, _) in self.active.items():
                    if off < o2 + b2 and o2 < off + ws_bytes:
                        self.errors.append(f"workspace [{off}, +{ws_bytes}) overlaps lane {other}")
                self.active[lane] = (off, ws_bytes, n)
                self.launches.append((time.monotonic(), lane, batch, off, ws_bytes))
                self.max_active_queries = max(self.max_active_queries,
                                              sum(a[2] for a in self.active.values()))
                self.max_active_lanes = max(self.max_active_lanes, len(self.active))
                self.lane_until[lane] = time.monotonic() + self.delay
                self.lane_fail[lane] = self.fail_poll_at == len(self.launches)
                if self.fail_launch_at == len(self.launches):
                    # fails after its work was enqueued: the lane stays busy
                    # with this workspace until quiesce() has waited for it
                    return rel.REL_EDEVICE
            return rel.REL_OK
        except Exception as e:  # reported by the test, never raised into C
            self.errors.append(repr(e))
            return rel.REL_EDEVICE

    def _quiesce(self, user, lane):
        with self.lock:
            until = self.lane_until[lane]
        if until is not None:
            time.sleep(max(0.0, until - time.monotonic()))
        with self.lock:
            self.lane_until[lane] = None
            self.active.pop(lane, None)
            self.quiesced.append(lane)

    def _poll(self, user, lane):
        with self.lock:
            if self.lane_until[lane] is None or time.monotonic() < self.lane_until[lane]:
                return 0
            self.lane_until[lane] = None
            self.active.pop(lane, None)
            return -rel.REL_EDEVICE if self.lane_fail[lane] else 1


def star(seed, n=3000):
    r = np.random.default_rng(seed)
    dim_key = r.permutation(500).astype(np.int32)
    region = r.integers(0, 25, size=500).astype(np.int32)
    fk = r.integers(0, 520, size=n).astype(np.int32)
    date = r.integers(0, 2557, size=n).astype(np.int32)
    price = r.integers(100, 10**7, size=n).astype(np.int64)
    return fk, date, price, dim_key, region


def query(data, lo, w, payload=True, max_groups=64):
    fk, date, price, dim_key, region = data
    dims = [dict(fk=0, key=dim_key, payload=region if payload else None)]
    keys = [("dim", 0)] if payload else []
    return HostPlan([fk, date, price], [(1, "range", lo, lo + w)], dims, keys,
                    [("sum", 2), ("count", None)], max_groups)


def make_server(ex, arena_bytes=1 << 30, max_slots=64, max_batch=8, lanes=2, open_lane_at=0):
    return serve.Server(arena_bytes, max_slots=max_slots, max_batch=max_batch, lanes=lanes,
                        open_lane_at=open_lane_at,
                        executor=ex.struct, arena_ptr=ARENA_BASE)


def wait_all(srv, n, timeout=30.0):
    got = {}
    end = time.monotonic() + timeout
    while len(got) < n and time.monotonic() < end:
        for c in srv.poll():
            assert c["ticket"] not in got, "a query completed twice"
            got[c["ticket"]] = c
        time.sleep(0.001)
    return got


def check_results(plans):
    for p in plans:
        want = oracle.pipeline(*p.spec)
        assert p.result is not None
        for a, b in zip(p.result[0] + p.result[1], want[0] + want[1]):
            assert np.array_equal(np.asarray(a), np.asarray(b))


def test_burst_is_batched_in_fifo_order_within_limits():
    data = star(1)
    plans = [query(data, 40 * i, 300 + i) for i in range(40)]
    ex = OracleExecutor(plans, lanes=2, delay=0.004)
    srv = make_server(ex, max_slots=12, max_batch=5, lanes=2)
    t_start = time.monotonic()
    tickets = [srv.submit(p) for p in plans]
    got = wait_all(srv, len(plans))
    assert srv.drain(10)
    t_end = time.monotonic()
    st = srv.stats()
    srv.close()
    assert not ex.errors, ex.errors
    assert sorted(got) == sorted(tickets)
    assert all(c["status"] == 0 for c in got.values())
    sizes = [len(b) for _, _, b, _, _ in ex.launches]
    assert max(sizes) <= 5 and sum(sizes) == 40
    assert max(sizes) > 1, "a burst must be batched"
    assert ex.max_active_queries <= 12 and ex.max_active_lanes <= 2
    order = [p for _, _, b, _, _ in ex.launches for p in b]
    assert order == plans, "queries of one shape launch in submission order"
    assert st["completed"] == 40 and st["batches"] == len(ex.launches)
    assert st["p50_ms"] is not None and st["p99_ms"] >= st["p50_ms"]
    # rows/s over the successful queries: 40 queries of 3000 fact rows, between
    # the first submission and the last completion (inside the measured span)
    assert 40 * 3000 / (t_end - t_start) <= st["rows_per_s"] < float("inf")
    check_results(plans)


def test_arena_budget_limits_admission():
    data = star(2)
    plans = [query(data, 30 * i, 200) for i in range(12)]
    one = rel.lib().rel_pipeline_batch_ws(ctypes.byref(plans[0].desc), 1)
    ex = OracleExecutor(plans, lanes=4, delay=0.003)
    # room for about two single-query workspaces at a time
    srv = make_server(ex, arena_bytes=int(2.2 * one), max_batch=8, lanes=4)
    for p in plans:
        srv.submit(p)
    got = wait_all(srv, len(plans))
    srv.close()
    assert not ex.errors, ex.errors
    assert len(got) == 12 and all(c["status"] == 0 for c in got.values())
    for _, _, b, off, nbytes in ex.launches:
        assert off + nbytes <= int(2.2 * one)
    assert max(len(b) for _, _, b, _, _ in ex.launches) <= 2
    check_results(plans)


def test_oversized_query_is_rejected_and_others_continue():
    data = star(3)
    small = [query(data, 100 * i, 500) for i in range(6)]
    fk, date, price, _, _ = data
    big_key = np.arange(2_000_000, dtype=np.int32)
    big = HostPlan([fk, date, price], [], [dict(fk=0, key=big_key, payload=big_key)],
                   [("dim", 0)], [("count", None)], 64)
    one = rel.lib().rel_pipeline_batch_ws(ctypes.byref(small[0].desc), 1)
    ex = OracleExecutor(small + [big], lanes=2)
    srv = make_server(ex, arena_bytes=4 * one, max_batch=2)
    tickets = [srv.submit(small[0]), srv.submit(small[1])]
    with pytest.raises(rel.RelError) as e:
        srv.submit(big)
    assert e.value.status == rel.REL_ENOMEM
    tickets += [srv.submit(p) for p in small[2:]]
    got = wait_all(srv, len(tickets))
    st = srv.stats()
    srv.close()
    assert not ex.errors, ex.errors
    assert sorted(got) == sorted(tickets) and all(c["status"] == 0 for c in got.values())
    assert st["rejected"] == 1
    check_results(small)


def test_shapes_are_never_mixed_in_a_batch():
    data = star(4)
    plans = [query(data, 50 * i, 400, payload=(i % 3 != 0)) for i in range(24)]
    ex = OracleExecutor(plans, lanes=1, delay=0.003)
    srv = make_server(ex, max_batch=6, lanes=1)
    for p in plans:
        srv.submit(p)
    got = wait_all(srv, len(plans))
    srv.close()
    assert not ex.errors, ex.errors
    assert len(got) == 24
    for _, _, b, _, _ in ex.launches:
        assert len({p.desc.dims[0].has_payload for p in b}) == 1
    check_results(plans)


def test_group_classes_are_never_mixed_in_a_batch():
    """Plans of one kernel shape but with max_groups in different classes
    (up to 4096, up to 65536, more) go to different batches."""
    data = star(4)
    classes = [64, 5000, 100_000]
    plans = [query(data, 50 * i, 400, max_groups=classes[i % 3]) for i in range(18)]
    ex = OracleExecutor(plans, lanes=1, delay=0.003)
    srv = make_server(ex, max_batch=6, lanes=1)
    for p in plans:
        srv.submit(p)
    got = wait_all(srv, len(plans))
    srv.close()
    assert not ex.errors, ex.errors
    assert len(got) == 18
    cls = lambda g: 0 if g <= 4096 else (1 if g <= 65536 else 2)
    assert any(len(b) > 1 for _, _, b, _, _ in ex.launches), "some batching happened"
    for _, _, b, _, _ in ex.launches:
        assert len({cls(p.desc.max_groups) for p in b}) == 1
    check_results(plans)


def test_forced_launch_failure_fails_only_that_batch(monkeypatch):
    monkeypatch.setenv("REL_FAULT", "launch:2")
    data = star(5)
    plans = [query(data, 60 * i, 300) for i in range(10)]
    ex = OracleExecutor(plans, lanes=1, delay=0.002)
    srv = make_server(ex, max_batch=3, lanes=1)
    tickets = [srv.submit(p) for p in plans]
    got = wait_all(srv, len(plans))
    st = srv.stats()
    srv.close()
    failed = [t for t in tickets if got[t]["status"] != 0]
    assert all(got[t]["status"] == rel.REL_EDEVICE for t in failed)
    # batch 1 ran, batch 2 was refused before running, the rest ran
    assert 1 <= len(failed) <= 3 and st["failed"] == len(failed)
    assert st["completed"] == 10 - len(failed)
    ran = {id(p) for _, _, b, _, _ in ex.launches for p in b}
    for t, p in zip(tickets, plans):
        assert (id(p) in ran) == (got[t]["status"] == 0)


def test_executor_failure_fails_only_that_batch():
    data = star(6)
    plans = [query(data, 60 * i, 300) for i in range(9)]
    ex = OracleExecutor(plans, lanes=1, delay=0.002, fail_poll_at=1)
    srv = make_server(ex, max_batch=3, lanes=1)
    tickets = [srv.submit(p) for p in plans]
    got = wait_all(srv, len(plans))
    srv.close()
    first = {id(p) for p in ex.launches[0][2]}
    for t, p in zip(tickets, plans):
        assert got[t]["status"] == (rel.REL_EDEVICE if id(p) in first else 0)


def test_invalid_plan_and_config_are_refused():
    data = star(7)
    p = query(data, 0, 100)
    ex = OracleExecutor([p], lanes=1)
    srv = make_server(ex, lanes=1)
    p.desc.n_aggs = 0
    with pytest.raises(rel.RelError) as e:
        srv.submit(p)
    assert e.value.status == rel.REL_EINVAL
    srv.close()
    with pytest.raises(rel.RelError):
        serve.Server(1 << 20, max_batch=0, executor=ex.struct, arena_ptr=ARENA_BASE)
    with pytest.raises(rel.RelError):
        serve.Server(1 << 20, executor=ex.struct, arena_ptr=ARENA_BASE + 8)


def test_poisson_arrivals_are_seeded():
    a = serve.poisson_arrivals(9, 2000, 500.0)
    b = serve.poisson_arrivals(9, 2000, 500.0)
    assert np.array_equal(a, b) and np.all(np.diff(a) > 0)
    # mean gap 1/qps within 10% over 2000 draws
    assert abs(a[-1] / 2000 - 1 / 500.0) < 0.1 / 500.0


def test_replay_reports_latency_on_a_trace():
    data = star(8)
    plans = [query(data, 13 * i, 250) for i in range(30)]
    ex = OracleExecutor(plans, lanes=2, delay=0.002)
    srv = make_server(ex, max_batch=4, lanes=2)
    res = serve.replay(srv, plans, serve.poisson_arrivals(10, 30, 2000.0))
    srv.close()
    assert not ex.errors, ex.errors
    assert res["ok"] == 30 and res["p99_ms"] >= res["p50_ms"] >= 2.0 - 0.5
    check_results(plans)


def test_second_lane_opens_only_for_a_backlog():
    """With a backlog threshold of 8 and one lane busy, a second starts only
    when 8 queries wait: three queries never run on two lanes at once."""
    data = star(5)
    plans = [query(data, 60 * i, 300) for i in range(3)]
    ex = OracleExecutor(plans, lanes=2, delay=0.01)
    srv = make_server(ex, max_batch=8, lanes=2, open_lane_at=8)
    for p in plans:
        srv.submit(p)
    got = wait_all(srv, len(plans))
    srv.close()
    assert not ex.errors, ex.errors
    assert len(got) == 3 and all(c["status"] == 0 for c in got.values())
    assert ex.max_active_lanes == 1
    check_results(plans)


def test_failed_launch_releases_its_workspace_only_after_quiesce():
    """A launch that fails after enqueueing work: the scheduler waits for the
    lane (executor quiesce) before the batch's arena block can be handed to
    another batch; the executor reports any workspace overlap with a lane
    whose work has not drained, and any launch on a lane still busy."""
    data = star(5)
    plans = [query(data, 30 * i, 200 + i) for i in range(12)]
    ex = OracleExecutor(plans, lanes=2, delay=0.02, fail_launch_at=1)
    srv = make_server(ex, max_slots=4, max_batch=2, lanes=2)
    tickets = [srv.submit(p) for p in plans]
    got = wait_all(srv, len(plans))
    assert srv.drain(10)
    st = srv.stats()
    srv.close()
    assert not ex.errors, ex.errors
    assert ex.quiesced and ex.quiesced[0] == ex.launches[0][1]
    first = {id(p) for p in ex.launches[0][2]}
    for t, p in zip(tickets, plans):
        assert (got[t]["status"] != 0) == (id(p) in first)
    assert st["failed"] == len(first) and st["completed"] == 12 - len(first)
    # the next batches reused the arena from offset 0 once the lane drained
    assert any(off == ex.launches[0][3] for _, _, _, off, _ in ex.launches[1:])
