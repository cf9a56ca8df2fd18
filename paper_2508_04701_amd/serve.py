"""Query serving over resident tables: a thin binding of rel_server_* of
include/rel.h (the scheduler, admission and batching are native) and a
replay driver for seeded arrival traces.

A query is a ``rel.Plan`` over device columns that stay allocated. The
server admits queries as lanes, slots and arena bytes free up and packs the
waiting ones into batches (continuous batching); each query completes once
its result rows are in its pinned host buffers.
"""

from __future__ import annotations

import ctypes
import time

import numpy as np
import torch

from . import rel

BATCH_WS = ctypes.CFUNCTYPE(ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int)
LAUNCH = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                          ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_size_t)
POLL = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int)
QUIESCE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int)


class Executor(ctypes.Structure):
    _fields_ = [("user", ctypes.c_void_p), ("batch_ws", BATCH_WS), ("launch", LAUNCH),
                ("poll", POLL), ("quiesce", QUIESCE)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t),
                ("max_slots", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("lanes", ctypes.c_int32), ("open_lane_at", ctypes.c_int32),
                ("executor", ctypes.POINTER(Executor))]


class Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("batch_size", ctypes.c_int32), ("t_submit_ns", ctypes.c_int64),
                ("t_launch_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64)]


class Counts(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "failed", "rejected",
                                              "batches", "batched_queries")]


def now_ns() -> int:
    return int(rel.lib().rel_server_now_ns())


class HostResult:
    """Pinned host buffers for one query's result rows (the plan's key and
    aggregate types, the plan's capacity)."""

    def __init__(self, plan):
        pin = torch.cuda.is_available()
        self.keys = [torch.empty(plan.cap, dtype=dt, pin_memory=pin) for dt in plan.key_dtypes]
        self.aggs = [torch.empty(plan.cap, dtype=torch.float64 if op == "avg" else torch.int64,
                                 pin_memory=pin) for op, _ in plan.aggs]
        self.count = torch.full((1,), -2, dtype=torch.int64, pin_memory=pin)
        self.outputs = rel.Outputs()
        for i, k in enumerate(self.keys):
            self.outputs.keys[i] = k.data_ptr()
        for i, a in enumerate(self.aggs):
            self.outputs.aggs[i] = a.data_ptr()
        self.outputs.cap = plan.cap
        self.outputs.d_groups = self.count.data_ptr()

    def result(self):
        n = int(self.count[0])
        if n < 0:
            raise rel.RelError(rel.REL_ECAPACITY, "more groups than max_groups")
        if n > len(self.aggs[0]):
            raise rel.RelError(rel.REL_ECAPACITY, f"{n} groups exceed the output capacity")
        return [k[:n] for k in self.keys], [a[:n] for a in self.aggs]


class Server:
    """rel_server over an arena of `arena_bytes` of device memory (the
    admission budget). ``max_batch=1, lanes=1`` serves one query at a time."""

    def __init__(self, arena_bytes: int, max_slots: int = 64, max_batch: int = 16,
                 lanes: int = 2, executor: Executor | None = None, arena_ptr: int | None = None,
                 open_lane_at: int = 0):
        self._executor = executor
        if arena_ptr is None:
            self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
            arena_ptr = self.arena.data_ptr()
        self.config = ServerConfig(arena_ptr, int(arena_bytes), max_slots, max_batch, lanes,
                                   open_lane_at,
                                   ctypes.pointer(executor) if executor is not None else None)
        h = ctypes.c_void_p()
        st = rel.lib().rel_server_create(ctypes.byref(self.config), ctypes.byref(h))
        if st != rel.REL_OK:
            raise rel.RelError(st, "rel_server_create failed")
        self._h = h
        self._queries = {}

    def submit(self, plan, host: HostResult | None = None) -> int:
        """Queues a plan; returns its ticket. The plan (and host buffers) are
        kept alive until the query completes."""
        t = ctypes.c_uint64()
        st = rel.lib().rel_server_submit(self._h, ctypes.byref(plan.desc),
                                         ctypes.byref(plan.outputs),
                                         ctypes.byref(host.outputs) if host is not None else None,
                                         ctypes.byref(t))
        if st != rel.REL_OK:
            raise rel.RelError(st, "query not admitted" if st == rel.REL_ENOMEM else
                               "query refused")
        self._queries[t.value] = (plan, host)
        return t.value

    def poll(self, max_items: int = 256) -> list:
        buf = (Completion * max_items)()
        n = rel.lib().rel_server_poll(self._h, buf, max_items)
        out = []
        for c in buf[:n]:
            self._queries.pop(c.ticket, None)
            out.append(dict(ticket=c.ticket, status=c.status, batch_size=c.batch_size,
                            t_submit_ns=c.t_submit_ns, t_launch_ns=c.t_launch_ns,
                            t_done_ns=c.t_done_ns))
        return out

    def drain(self, timeout_s: float = 60.0) -> bool:
        return rel.lib().rel_server_drain(self._h, int(timeout_s * 1000)) == rel.REL_OK

    def stats(self) -> dict:
        c = Counts()
        p50, p99 = ctypes.c_int64(), ctypes.c_int64()
        rate = ctypes.c_double()
        rel.lib().rel_server_stats(self._h, ctypes.byref(c), ctypes.byref(p50), ctypes.byref(p99),
                                   ctypes.byref(rate))
        d = {n: getattr(c, n) for n, _ in Counts._fields_}
        d["rows_per_s"] = rate.value
        d["p50_ms"] = p50.value / 1e6 if p50.value >= 0 else None
        d["p99_ms"] = p99.value / 1e6 if p99.value >= 0 else None
        return d

    def close(self):
        if self._h:
            rel.lib().rel_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def poisson_arrivals(seed: int, n: int, qps: float) -> np.ndarray:
    """Arrival offsets (seconds) of a seeded Poisson process of rate qps:
    cumulative exponential gaps drawn by inversion of counter-based uniforms."""
    from . import datagen
    u = (datagen.raw_u64(seed, 60, n) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.cumsum(-np.log1p(-u) / qps)


def replay(server: Server, plans, arrivals: np.ndarray, hosts: list | None = None,
           on_done=None) -> dict:
    """Submits query i at arrivals[i] seconds after the start, collecting
    completions meanwhile; returns per-query latency statistics (scheduled
    arrival -> done on the server clock, so a late submission counts against
    the query) and the wall time from the start to the last completion.

    plans: a list of plans (with `hosts` their host buffers), or a callable
    make(i) -> (plan, host) or None when query i cannot be formed yet (it is
    retried); on_done(i, completion) is called as each query completes."""
    n = len(arrivals)
    make = plans if callable(plans) else (lambda i: (plans[i], hosts[i] if hosts else None))
    t0 = now_ns() + 2_000_000
    due = t0 + (np.asarray(arrivals) * 1e9).astype(np.int64)
    done = {}
    index = {}
    tickets = [None] * n
    i = 0
    while i < n or len(done) < n:
        now = now_ns()
        while i < n and due[i] <= now:
            q = make(i)
            if q is None:
                break
            tickets[i] = server.submit(q[0], q[1])
            index[tickets[i]] = i
            i += 1
        for c in server.poll():
            done[c["ticket"]] = c
            if on_done is not None:
                on_done(index[c["ticket"]], c)
        if i < n and due[i] - now_ns() > 200_000:
            time.sleep(50e-6)
    lat = np.array([done[t]["t_done_ns"] - due[k] for k, t in enumerate(tickets)], np.int64)
    status = np.array([done[t]["status"] for t in tickets])
    batch = np.array([done[t]["batch_size"] for t in tickets])
    wall = max(c["t_done_ns"] for c in done.values()) - t0
    ok = lat[status == 0]
    pct = (lambda q: float(np.percentile(ok, q, method="inverted_cdf")) / 1e6) if len(ok) else \
        (lambda q: None)
    return dict(n=n, ok=int((status == 0).sum()), wall_s=wall / 1e9, p50_ms=pct(50),
                p99_ms=pct(99), max_ms=float(ok.max()) / 1e6 if len(ok) else None,
                mean_batch=float(batch.mean()), tickets=tickets)
